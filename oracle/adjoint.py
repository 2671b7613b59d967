"""Gradient of a terminal objective of the WADG sweep -- oracle (test
infrastructure; plain FP64 NumPy, dense matrices, small meshes only).

The sensitivity problem: a state y0 = (p0, u0, v0) is advanced by n LSRK
steps of the WADG scheme with wave speed c^2 = gamma c0^2(x), and

    J(y0, gamma) = sum over all nodal pressure values (p(T) - p_target)^2.

Two routes, both plain and both different from the GPU's:

* ``gradient`` -- from the definitions.  The semi-discrete operator is
  linear, dQ/dt = L Q, and c^2 enters it only through the pressure mass
  inverse M_{c^2/J} (Section 7), linearly, so L(gamma) = E(gamma) L_1 with
  E = diag(gamma on the p rows, 1 on the u, v rows) and L_1 the operator at
  gamma = 1 (assembled densely from the oracle's right-hand side).  One
  step of the LSRK scheme (Section 5.2) on a linear autonomous system is
  Phi = R(dt L), R the stability polynomial, so
      dJ/dy0    = (Phi^T)^n g,   g = dJ/dq(T) = 2 (p(T) - p_target) on p,
      dJ/dgamma = g . qdot_n,    qdot_{m+1} = Phi qdot_m + Phidot q_m,
  the forward (tangent-linear) sensitivity, with
      Phidot = sum_k R_k dt^k sum_{j<k} L^j Ldot L^{k-1-j},  Ldot = E_p L_1.
* ``gradient_reverse`` -- the reverse sweep of the 2N-storage recursion
  itself (res <- A_i res + dt L y; y <- y + B_i res), stage by stage, with
  the dense transpose L^T: per stage, in reverse,
      rbar += B_i ybar;  gammabar += dt rbar . Ldot y_{i-1};
      ybar += dt L^T rbar;  rbar *= A_i.
  The GPU runs this recursion; the oracle checks it against ``gradient``.

State vectors are nodal, ordered like [3][Np][K] (field, node, element).
"""

import numpy as np

from .lsrk import LSRK54, stability_polynomial_coeffs
from .wadg import WADGOracle


def step_matrix(L, dt):
    """Phi = R(dt L) = sum_k R_k (dt L)^k."""
    coeffs = [float(c) for c in stability_polynomial_coeffs()]
    n = L.shape[0]
    Z = dt * L
    term = np.eye(n)
    phi = coeffs[0] * term
    for c in coeffs[1:]:
        term = term @ Z
        phi = phi + c * term
    return phi


def step_matrix_derivative(L, Ld, dt):
    """d/dgamma R(dt L(gamma)) for dL/dgamma = Ld (matrices need not commute)."""
    coeffs = [float(c) for c in stability_polynomial_coeffs()]
    n = L.shape[0]
    pows = [np.eye(n)]
    for _ in range(len(coeffs) - 2):
        pows.append(pows[-1] @ L)
    out = np.zeros((n, n))
    for k in range(1, len(coeffs)):
        s = sum(pows[j] @ Ld @ pows[k - 1 - j] for j in range(k))
        out += coeffs[k] * dt ** k * s
    return out


class TerminalObjective:
    """J(y0, gamma) for one mesh, base wave speed c0^2 and penalties."""

    def __init__(self, mesh, c0=None, nq1=None, tau_p=1.0, tau_u=1.0):
        self.c0 = (lambda x, y: np.ones_like(x)) if c0 is None else c0
        self.o1 = WADGOracle(mesh, nq1=nq1, c2=self.c0, tau_p=tau_p, tau_u=tau_u)
        self.shape = (3, self.o1.Np, self.o1.K)
        n = int(np.prod(self.shape))
        self.L1 = self.o1.assemble()
        self.p_rows = np.zeros(n)
        self.p_rows[: self.o1.Np * self.o1.K] = 1.0

    def operator(self, gamma):
        return (1.0 + (gamma - 1.0) * self.p_rows)[:, None] * self.L1

    def operator_derivative(self):
        return self.p_rows[:, None] * self.L1

    def _seed(self, qT, p_target):
        g = np.zeros_like(qT)
        np.copyto(g[: self.o1.Np * self.o1.K], 2.0 * (qT[: self.o1.Np * self.o1.K]
                                                      - np.ravel(p_target)))
        return g

    def value(self, y0, p_target, gamma, dt, nsteps):
        """J by the oracle's own stepper (the WADG sweep with c^2 = gamma c0^2)."""
        o = WADGOracle(self.o1.mesh, nq1=self.o1.nq1, c2=lambda x, y: gamma * self.c0(x, y),
                       tau_p=self.o1.tau_p, tau_u=self.o1.tau_u)
        qT = o.integrate(np.asarray(y0, dtype=np.float64).reshape(self.shape), dt, nsteps)
        return float(np.sum((qT[0] - np.asarray(p_target).reshape(qT[0].shape)) ** 2))

    def gradient(self, y0, p_target, gamma, dt, nsteps):
        """(J, dJ/dy0 [3][Np][K], dJ/dgamma) by the transposed step matrix and
        the tangent-linear recursion."""
        L = self.operator(gamma)
        phi = step_matrix(L, dt)
        phid = step_matrix_derivative(L, self.operator_derivative(), dt)
        q = np.asarray(y0, dtype=np.float64).reshape(-1)
        qdot = np.zeros_like(q)
        for _ in range(nsteps):
            qdot = phi @ qdot + phid @ q
            q = phi @ q
        g = self._seed(q, p_target)
        J = float(np.sum((q[: self.o1.Np * self.o1.K] - np.ravel(p_target)) ** 2))
        lam = g
        for _ in range(nsteps):
            lam = phi.T @ lam
        return J, lam.reshape(self.shape), float(g @ qdot)

    def adjoint_apply(self, w, gamma, dt, nsteps):
        """(Phi^T)^n w: the transposed sweep applied to any seed w."""
        phi = step_matrix(self.operator(gamma), dt)
        lam = np.asarray(w, dtype=np.float64).reshape(-1)
        for _ in range(nsteps):
            lam = phi.T @ lam
        return lam.reshape(self.shape)

    def gradient_reverse(self, y0, p_target, gamma, dt, nsteps):
        """The same gradient by the reverse sweep of the 2N-storage stages."""
        L = self.operator(gamma)
        Ld = self.operator_derivative()
        A, B = LSRK54.A, LSRK54.B
        q = np.asarray(y0, dtype=np.float64).reshape(-1)
        inputs = []
        for _ in range(nsteps):
            res = np.zeros_like(q)
            ys = []
            for i in range(5):
                ys.append(q)
                res = A[i] * res + dt * (L @ q)
                q = q + B[i] * res
            inputs.append(ys)
        J = float(np.sum((q[: self.o1.Np * self.o1.K] - np.ravel(p_target)) ** 2))
        ybar = self._seed(q, p_target)
        gbar = 0.0
        for ys in reversed(inputs):
            rbar = np.zeros_like(q)
            for i in reversed(range(5)):
                rbar = rbar + B[i] * ybar
                gbar += dt * float(rbar @ (Ld @ ys[i]))
                ybar = ybar + dt * (L.T @ rbar)
                rbar = A[i] * rbar
        return J, ybar.reshape(self.shape), gbar
