"""Reference square [-1,1]^2 with the tensor space Q^N (paper, Section 2).

The oracle works in the orthonormal Legendre basis
``phi_{i + (N+1) j}(r, s) = L_i(r) L_j(s)``, ``L_m = sqrt((2m+1)/2) P_m``,
so the reference mass matrix is the identity.  The nodal Gauss-Lobatto
points are only the input/output format.
"""

import numpy as np


def legendre_orthonormal(nmax, x):
    """Values and first derivatives of L_0..L_nmax at points x.

    Uses the three-term recurrence (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}
    and P'_{n+1} = P'_{n-1} + (2n+1) P_n.  Returns two arrays [nmax+1][len(x)].
    """
    x = np.asarray(x, dtype=np.float64)
    P = np.zeros((nmax + 1,) + x.shape)
    dP = np.zeros_like(P)
    P[0] = 1.0
    if nmax >= 1:
        P[1] = x
        dP[1] = 1.0
    for n in range(1, nmax):
        P[n + 1] = ((2 * n + 1) * x * P[n] - n * P[n - 1]) / (n + 1)
        dP[n + 1] = dP[n - 1] + (2 * n + 1) * P[n]
    scale = np.sqrt((2 * np.arange(nmax + 1) + 1) / 2.0).reshape((-1,) + (1,) * x.ndim)
    return P * scale, dP * scale


def gauss_legendre(n):
    """n-point Gauss-Legendre rule on [-1,1] (exact to degree 2n-1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return x.astype(np.float64), w.astype(np.float64)


def gll_nodes(N):
    """Gauss-Lobatto-Legendre nodes: -1, 1 and the N-1 roots of P_N'.

    Newton's method on P_N' from the Chebyshev-Lobatto guesses -cos(pi i/N),
    with P_N'' from Legendre's equation (1-x^2) P'' = 2x P' - N(N+1) P.
    """
    x = -np.cos(np.pi * np.arange(N + 1) / N)
    inner = x[1:-1].copy()
    for _ in range(100):
        P, dP = legendre_orthonormal(N, inner)
        p, dp = P[N], dP[N]
        d2p = (2 * inner * dp - N * (N + 1) * p) / (1 - inner ** 2)
        step = dp / d2p
        inner = inner - step
        if np.all(np.abs(step) < 1e-16):
            break
    x[1:-1] = inner
    x[0], x[-1] = -1.0, 1.0
    return 0.5 * (x - x[::-1])


class ReferenceQuad:
    """Reference-element operators for degree N and an nq1-point Gauss rule.

    Quadrature points are indexed q = qi + nq1 * qj (r index fastest); modes
    m = i + (N+1) j; GLL nodes n = a + (N+1) b.  Faces (parameter in
    brackets): 0: s=-1 (r), 1: r=+1 (s), 2: s=+1 (r), 3: r=-1 (s).
    """

    def __init__(self, N, nq1):
        self.N, self.nq1 = N, nq1
        Np1 = N + 1
        self.Np = Np1 * Np1
        t, w = gauss_legendre(nq1)
        self.t1, self.w1 = t, w
        L, dL = legendre_orthonormal(N, t)                 # [Np1][nq1]

        def tensor(A, B):
            """A: [Np1][na] over r, B: [Np1][nb] over s -> [point][mode] with
            point qi + na*qj and mode i + Np1*j."""
            return np.einsum("ip,jq->qpji", A, B).reshape(A.shape[1] * B.shape[1], Np1 * Np1)

        self.V = tensor(L, L)             # phi_m at volume points
        self.Vr = tensor(dL, L)           # d/dr
        self.Vs = tensor(L, dL)           # d/ds
        self.W = np.outer(w, w).reshape(-1)   # symmetric in (qi, qj)
        rq = np.tile(t, nq1)
        sq = np.repeat(t, nq1)
        self.rq, self.sq = rq, sq

        # GLL nodes and the nodal <-> modal Vandermonde
        g = gll_nodes(N)
        self.gll = g
        Lg, _ = legendre_orthonormal(N, g)
        self.Vn = tensor(Lg, Lg)          # [node][mode]

        # face points in reference coordinates, parameter order
        one = np.ones(nq1)
        self.face_rs = [(t, -one), (one, t), (t, one), (-one, t)]
        self.Vf, self.Vfr, self.Vfs = [], [], []
        for (r, s) in self.face_rs:
            Lr, dLr = legendre_orthonormal(N, r)
            Ls, dLs = legendre_orthonormal(N, s)
            # modes m = i + Np1 j evaluated at points along the face
            self.Vf.append(np.einsum("ip,jp->pji", Lr, Ls).reshape(nq1, -1))
            self.Vfr.append(np.einsum("ip,jp->pji", dLr, Ls).reshape(nq1, -1))
            self.Vfs.append(np.einsum("ip,jp->pji", Lr, dLs).reshape(nq1, -1))
        self.wf = w
        # reference mass matrix, by quadrature (identity up to rounding)
        self.Mhat = self.V.T @ (self.W[:, None] * self.V)
