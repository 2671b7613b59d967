"""Periodic curvilinear quadrilateral meshes (inputs only).

The mesh is the unit torus [0,1)^2 split into ``K1D x K1D`` cells, each cell
mapped by the smooth periodic warp

    Phi(xi, eta) = (xi, eta) + eps * sin(2 pi xi) * sin(2 pi eta) * (1, 1),

whose Jacobian is ``1 + 2 pi eps sin(2 pi (xi + eta))`` (``warp="diag"``, the
default).  Because this warp moves x and y by the same amount, the
interpolated map has y - x affine on every element, and its Jacobian lies in
Q^N.  ``warp="skew"`` displaces y by ``eps sin(2 pi xi) sin(4 pi eta)``
instead, which gives a Jacobian outside Q^N.  Elements are
isoparametric (the paper restricts itself to isoparametric maps, Section 1):
each element is described by the physical coordinates of its (N+1)^2
Gauss-Lobatto-Legendre nodes, and the element map is the degree-N
interpolant of those nodes.  Adjacent elements share the GLL nodes of their
common face, so the mesh is conforming.

Optionally every element's local reference frame is rotated by a seeded
multiple of 90 degrees; neighbouring faces then run in opposite directions
and the connectivity carries a flip bit.  The discrete solution does not
depend on the local frames, which makes this a useful connectivity test.

Face numbering of the reference square [-1,1]^2 (parameter direction in
brackets): 0: s=-1 (r increasing), 1: r=+1 (s increasing), 2: s=+1 (r
increasing), 3: r=-1 (s increasing).  ``etof[k][f] = f_nbr | (flip << 2)``
where ``flip`` means that the neighbour traverses the shared face in the
opposite direction.
"""

from dataclasses import dataclass

import numpy as np
from numpy.polynomial import legendre as npleg


def gll_points(N):
    """Gauss-Lobatto-Legendre points on [-1,1]: the end points and the roots of
    P_N'.  These are the node positions of the nodal input/output format."""
    if N < 1:
        raise ValueError("N must be >= 1")
    inner = npleg.Legendre.basis(N).deriv().roots() if N > 1 else np.zeros(0)
    pts = np.concatenate(([-1.0], np.sort(np.real(inner)), [1.0]))
    # symmetrise exactly so that the node set is closed under x -> -x
    pts = 0.5 * (pts - pts[::-1])
    return pts


@dataclass
class QuadMesh:
    N: int
    K1D: int
    eps: float
    x: np.ndarray      # [K][Np] physical x of GLL nodes, node n = a + (N+1) b
    y: np.ndarray      # [K][Np]
    etoe: np.ndarray   # [K][4] int32 neighbour element across each local face
    etof: np.ndarray   # [K][4] int32 neighbour local face | (flip << 2)
    rot: np.ndarray    # [K] int32 local-frame rotation (multiples of 90 degrees)

    @property
    def K(self):
        return self.x.shape[0]

    @property
    def Np(self):
        return (self.N + 1) ** 2


def _rotate_index(rho, a, b, N):
    """Local node (a, b) -> node of the unrotated frame, for a frame rotated by
    rho * 90 degrees: (r, s) -> (-s, r) applied rho times.  GLL points are
    symmetric, so a rotation maps the node lattice onto itself."""
    for _ in range(rho % 4):
        a, b = N - b, a
    return a, b


def _rotate_corner(rho, r, s):
    for _ in range(rho % 4):
        r, s = -s, r
    return r, s


# local face -> (start corner, end corner) in parameter order
_FACE_CORNERS = {0: ((-1, -1), (1, -1)), 1: ((1, -1), (1, 1)),
                 2: ((-1, 1), (1, 1)), 3: ((-1, -1), (-1, 1))}
# unrotated faces: which coordinate is constant, its value, parameter axis
_BASE_FACE = {(1, -1): 0, (0, 1): 1, (1, 1): 2, (0, -1): 3}
_BASE_NBR = {0: (0, -1, 2), 1: (1, 0, 3), 2: (0, 1, 0), 3: (-1, 0, 1)}


def _face_in_base(rho, f):
    """Which unrotated face local face ``f`` lies on, and whether the local
    parameter runs in the unrotated face's parameter direction."""
    (r0, s0), (r1, s1) = _FACE_CORNERS[f]
    R0, S0 = _rotate_corner(rho, r0, s0)
    R1, S1 = _rotate_corner(rho, r1, s1)
    if R0 == R1:          # r' constant -> face 1 or 3, parameter s'
        bf = _BASE_FACE[(0, R0)]
        forward = S1 > S0
    else:                 # s' constant -> face 0 or 2, parameter r'
        bf = _BASE_FACE[(1, S0)]
        forward = R1 > R0
    return bf, forward


def periodic_quad_mesh(K1D, N, eps=0.05, rotate_seed=None, warp="diag"):
    """Build the periodic warped ``K1D x K1D`` mesh of degree-``N`` elements.

    Element ``k = i + K1D * j`` covers cell (i, j).  With ``rotate_seed`` set,
    each element's local frame is rotated by ``rng.integers(0, 4)`` quarter
    turns (numpy default_rng(rotate_seed), one draw per element in order k).
    """
    if K1D < 2:
        raise ValueError("K1D must be >= 2 for a periodic mesh")
    Np1 = N + 1
    K = K1D * K1D
    r = gll_points(N)
    if rotate_seed is None:
        rot = np.zeros(K, dtype=np.int32)
    else:
        rot = np.random.default_rng(rotate_seed).integers(0, 4, size=K).astype(np.int32)

    # node coordinates: unrotated lattice first, then each element's rotation
    ii, jj = np.meshgrid(np.arange(K1D), np.arange(K1D), indexing="xy")
    ii = ii.reshape(K, 1).astype(float)          # k = i + K1D * j
    jj = jj.reshape(K, 1).astype(float)
    aa = np.tile(np.arange(Np1), Np1)            # base node n = a + Np1 * b
    bb = np.repeat(np.arange(Np1), Np1)
    xi = (ii + 0.5 * (1.0 + r[aa])) / K1D
    eta = (jj + 0.5 * (1.0 + r[bb])) / K1D
    g = eps * np.sin(2 * np.pi * xi) * np.sin(2 * np.pi * eta)
    if warp == "diag":
        xb, yb = xi + g, eta + g
    elif warp == "skew":
        xb = xi + g
        yb = eta + eps * np.sin(2 * np.pi * xi) * np.sin(4 * np.pi * eta)
    else:
        raise ValueError(warp)
    node_map = np.empty((4, Np1 * Np1), dtype=np.int64)
    for rho in range(4):
        for b in range(Np1):
            for a in range(Np1):
                ab, bb_ = _rotate_index(rho, a, b, N)
                node_map[rho, a + Np1 * b] = ab + Np1 * bb_
    sel = node_map[rot]                          # [K][Np] base index per local node
    x = np.take_along_axis(xb, sel, axis=1)
    y = np.take_along_axis(yb, sel, axis=1)

    face_tab = [[_face_in_base(rho, f) for f in range(4)] for rho in range(4)]
    local_of_base = [{face_tab[rho][f][0]: f for f in range(4)} for rho in range(4)]
    etoe = np.empty((K, 4), dtype=np.int32)
    etof = np.empty((K, 4), dtype=np.int32)
    for j in range(K1D):
        for i in range(K1D):
            k = i + K1D * j
            rk = int(rot[k])
            for f in range(4):
                bf, fwd = face_tab[rk][f]
                di, dj, bf_nbr = _BASE_NBR[bf]
                kn = ((i + di) % K1D) + K1D * ((j + dj) % K1D)
                rn = int(rot[kn])
                fn = local_of_base[rn][bf_nbr]
                fwd_n = face_tab[rn][fn][1]
                etoe[k, f] = kn
                etof[k, f] = fn | (int(fwd != fwd_n) << 2)
    return QuadMesh(N=N, K1D=K1D, eps=eps, x=x, y=y, etoe=etoe, etof=etof, rot=rot)


def periodic_cover(mesh, m):
    """The ``m x m`` periodic cover of a periodic mesh: ``m^2`` copies of
    ``mesh`` side by side, joined into one torus of ``(m K1D)^2`` elements.

    Every copy keeps the base mesh's node coordinates unchanged (faces match
    modulo the unit period, as on the base torus's own wrap-around faces),
    its local frames and face flips.  Element ``k = I + (m K1D) J`` is a copy
    of base element ``base[k] = (I mod K1D) + K1D (J mod K1D)``; its neighbour
    across face f is the element displaced from (I, J) as the base neighbour
    is displaced from the base element.  A state that repeats the base state
    on every copy therefore evolves as the base state does, copy by copy.
    Returns ``(cover, base)``.  Needs ``mesh.K1D >= 3`` (so that neighbour
    displacements are unambiguous)."""
    K1D = int(mesh.K1D)
    m = int(m)
    if K1D < 3 or m < 1:
        raise ValueError("periodic_cover needs K1D >= 3 and m >= 1")
    C1D = m * K1D
    k = np.arange(C1D * C1D, dtype=np.int64)
    I, J = k % C1D, k // C1D
    base = (I % K1D) + K1D * (J % K1D)
    kb_n = mesh.etoe.astype(np.int64)                   # [Kb][4]
    di = (kb_n % K1D - (np.arange(mesh.K) % K1D)[:, None] + 1) % K1D - 1
    dj = (kb_n // K1D - (np.arange(mesh.K) // K1D)[:, None] + 1) % K1D - 1
    etoe = ((I[:, None] + di[base]) % C1D + C1D * ((J[:, None] + dj[base]) % C1D))
    cover = QuadMesh(N=mesh.N, K1D=C1D, eps=mesh.eps, x=mesh.x[base], y=mesh.y[base],
                     etoe=etoe.astype(np.int32), etof=mesh.etof[base], rot=mesh.rot[base])
    return cover, base
