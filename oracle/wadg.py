"""Weight-adjusted DG for the acoustic wave equation on curvilinear quads --
the oracle (test infrastructure; plain FP64 NumPy, modal basis).

What is computed, and where the paper defines it:

* Semi-discrete system M dQ/dt = A_h Q with block-diagonal mass M_{J^k}
  (Section 4, opening).  Here ``b = A_h Q`` is the weak-form load vector.
* Right-hand side: the strong-weak form of Section 4.1 with rho = 1,
  jump [u] = u^+ - u^-, average {u} = (u^+ + u^-)/2, outward normal n = n^-:
      (1/c^2) p_t :  int_D u . grad(v) J  -  int_dD 1/2 (2 {u}.n - tau_p [p]) v sJ
      u_t         : -int_D grad(p) . tau J - int_dD 1/2 ([p] - tau_u [u].n) tau.n sJ
  Volume integrals use an nq1 x nq1 Gauss rule, faces an nq1-point Gauss
  rule.  Geometric factors come from the isoparametric map (Section 1;
  Section 4.1 on geometric factors of polynomial maps).
* WADG mass inverse (Section 4, the weight-adjusted approximation):
      M_{J}^{-1}      ~ Mhat^{-1} M_{1/J} Mhat^{-1}       (velocity)
      M_{J/c^2}^{-1}  ~ Mhat^{-1} M_{c^2/J} Mhat^{-1}     (pressure, Section 7)
  with M_w = V_q^T diag(w_q W_q) V_q formed explicitly per element.
* Exact curvilinear DG comparator: M_{J/c^2}^{-1}, M_J^{-1} by dense solves
  (Section 4: what WADG avoids storing).
* LSRK(5,4) time stepping (``lsrk``), slices advanced one after another.

Periodic meshes only (the Dirichlet mirror of Section 4.1 does not arise).
"""

import numpy as np

from .basis import ReferenceQuad
from .lsrk import lsrk_integrate


class WADGOracle:
    def __init__(self, mesh, nq1=None, c2=None, tau_p=1.0, tau_u=1.0, check_mesh=True):
        self.mesh = mesh
        self.N = N = mesh.N
        self.nq1 = nq1 = (N + 2) if nq1 is None else nq1
        self.ref = ref = ReferenceQuad(N, nq1)
        self.K = K = mesh.K
        self.Np = ref.Np
        self.tau_p, self.tau_u = float(tau_p), float(tau_u)

        # modal coefficients of the isoparametric element map: x_nodes = Vn c
        self.Vn_inv = np.linalg.inv(ref.Vn)
        self.cx = mesh.x @ self.Vn_inv.T          # [K][Np]
        self.cy = mesh.y @ self.Vn_inv.T

        # volume geometry at quadrature points
        xr, xs = self.cx @ ref.Vr.T, self.cx @ ref.Vs.T
        yr, ys = self.cy @ ref.Vr.T, self.cy @ ref.Vs.T
        J = xr * ys - xs * yr
        if np.any(~np.isfinite(J)) or np.any(J <= 0):
            raise ValueError("non-positive or non-finite Jacobian")
        self.J = J
        rx, ry, sx, sy = ys / J, -xs / J, -yr / J, xr / J
        self.xq, self.yq = self.cx @ ref.V.T, self.cy @ ref.V.T
        c2 = (lambda x, y: np.ones_like(x)) if c2 is None else c2
        self.c2q = np.asarray(c2(self.xq, self.yq), dtype=np.float64)
        if np.any(self.c2q <= 0):
            raise ValueError("c^2 must be positive")
        # physical gradient of each basis function at each quadrature point
        self.Dx = rx[:, :, None] * ref.Vr[None] + sx[:, :, None] * ref.Vs[None]
        self.Dy = ry[:, :, None] * ref.Vr[None] + sy[:, :, None] * ref.Vs[None]
        self.WJ = ref.W[None, :] * J

        # face geometry: outward normal times surface Jacobian
        self.nx, self.ny, self.sJ, self.xf, self.yf = [], [], [], [], []
        for f in range(4):
            fxr, fxs = self.cx @ ref.Vfr[f].T, self.cx @ ref.Vfs[f].T
            fyr, fys = self.cy @ ref.Vfr[f].T, self.cy @ ref.Vfs[f].T
            if f == 0:
                ax, ay = fyr, -fxr
            elif f == 1:
                ax, ay = fys, -fxs
            elif f == 2:
                ax, ay = -fyr, fxr
            else:
                ax, ay = -fys, fxs
            sJ = np.hypot(ax, ay)
            self.nx.append(ax / sJ)
            self.ny.append(ay / sJ)
            self.sJ.append(sJ)
            self.xf.append(self.cx @ ref.Vf[f].T)
            self.yf.append(self.cy @ ref.Vf[f].T)

        # neighbour of each face point: element, face, point index
        self.nbr_k = mesh.etoe.astype(np.int64)
        self.nbr_f = (mesh.etof & 3).astype(np.int64)
        flip = (mesh.etof >> 2) & 1
        j = np.arange(nq1)
        self.nbr_j = np.where(flip[:, :, None] == 1, nq1 - 1 - j[None, None, :],
                              j[None, None, :])      # [K][4][nq1]
        if check_mesh:
            self._check_conforming()

        # WADG inverse-mass operators, one explicit Np x Np matrix per element
        Minv = np.linalg.inv(ref.Mhat)
        Mw_p = np.einsum("qi,kq,qj->kij", ref.V, ref.W[None] * self.c2q / J, ref.V)
        Mw_u = np.einsum("qi,kq,qj->kij", ref.V, ref.W[None] / J, ref.V)
        self.Wp = Minv[None] @ Mw_p @ Minv[None]
        self.Wu = Minv[None] @ Mw_u @ Minv[None]
        self.Mw_p, self.Mw_u, self.Minv = Mw_p, Mw_u, Minv
        # exact curvilinear-DG mass matrices (comparator)
        self.M_Jc2 = np.einsum("qi,kq,qj->kij", ref.V, ref.W[None] * J / self.c2q, ref.V)
        self.M_J = np.einsum("qi,kq,qj->kij", ref.V, ref.W[None] * J, ref.V)

    # ------------------------------------------------------------------ mesh
    def _check_conforming(self):
        """Matched face points must coincide (modulo the unit period)."""
        for f in range(4):
            kn, fn, jn = self.nbr_k[:, f], self.nbr_f[:, f], self.nbr_j[:, f, :]
            xo = np.stack(self.xf)[fn[:, None], kn[:, None], jn]
            yo = np.stack(self.yf)[fn[:, None], kn[:, None], jn]
            dx, dy = xo - self.xf[f], yo - self.yf[f]
            err = max(np.max(np.abs(dx - np.round(dx))), np.max(np.abs(dy - np.round(dy))))
            if err > 1e-9:
                raise ValueError(f"mesh faces do not conform (face {f}, err {err:.2e})")

    # ----------------------------------------------------- nodal <-> modal
    def to_modal(self, Qn):
        """[3][Np][K] nodal (GLL) -> [3][K][Np] modal coefficients."""
        return np.stack([np.asarray(Qn[f]).T @ self.Vn_inv.T for f in range(3)])

    def to_nodal(self, Qm):
        """[3][K][Np] modal -> [3][Np][K] nodal."""
        return np.stack([(Qm[f] @ self.ref.Vn.T).T for f in range(3)])

    # ------------------------------------------------------------- rhs
    def load_vector(self, Qm):
        """b = A_h Q for modal Q [3][K][Np]: the strong-weak form, Section 4.1."""
        ref = self.ref
        P, U, V = Qm
        uq, vq = U @ ref.V.T, V @ ref.V.T
        px = np.einsum("kqm,km->kq", self.Dx, P)
        py = np.einsum("kqm,km->kq", self.Dy, P)
        # volume: (u . grad v) J and -(grad p . tau) J
        bp = (np.einsum("kqm,kq->km", self.Dx, self.WJ * uq)
              + np.einsum("kqm,kq->km", self.Dy, self.WJ * vq))
        bu = -(self.WJ * px) @ ref.V
        bv = -(self.WJ * py) @ ref.V
        # surface: traces on every face, own (minus) and neighbour (plus)
        tr = np.stack([np.stack([F @ ref.Vf[f].T for F in (P, U, V)]) for f in range(4)])
        for f in range(4):
            kn, fn, jn = self.nbr_k[:, f], self.nbr_f[:, f], self.nbr_j[:, f, :]
            pm, um, vm = tr[f]
            pp = tr[fn[:, None], 0, kn[:, None], jn]
            up = tr[fn[:, None], 1, kn[:, None], jn]
            vp = tr[fn[:, None], 2, kn[:, None], jn]
            nx, ny = self.nx[f], self.ny[f]
            jump_p = pp - pm
            avg_un = 0.5 * ((up + um) * nx + (vp + vm) * ny)
            jump_un = (up - um) * nx + (vp - vm) * ny
            flux_p = 0.5 * (2.0 * avg_un - self.tau_p * jump_p)
            flux_u = 0.5 * (jump_p - self.tau_u * jump_un)
            wsJ = ref.wf[None, :] * self.sJ[f]
            bp = bp - (wsJ * flux_p) @ ref.Vf[f]
            bu = bu - (wsJ * flux_u * nx) @ ref.Vf[f]
            bv = bv - (wsJ * flux_u * ny) @ ref.Vf[f]
        return np.stack([bp, bu, bv])

    def apply_mass_inverse(self, b, mass="wadg"):
        """M^{-1} b per element: WADG (default) or exact curvilinear DG."""
        if mass == "wadg":
            return np.stack([np.einsum("kij,kj->ki", self.Wp, b[0]),
                             np.einsum("kij,kj->ki", self.Wu, b[1]),
                             np.einsum("kij,kj->ki", self.Wu, b[2])])
        if mass == "dg":
            return np.stack([np.linalg.solve(self.M_Jc2, b[0][..., None])[..., 0],
                             np.linalg.solve(self.M_J, b[1][..., None])[..., 0],
                             np.linalg.solve(self.M_J, b[2][..., None])[..., 0]])
        raise ValueError(mass)

    def rhs_modal(self, Qm, mass="wadg"):
        return self.apply_mass_inverse(self.load_vector(Qm), mass)

    def rhs(self, Q, mass="wadg"):
        """dQ/dt for nodal states [S][3][Np][K] (or one slice [3][Np][K])."""
        Q = np.asarray(Q, dtype=np.float64)
        if Q.ndim == 3:
            return self.to_nodal(self.rhs_modal(self.to_modal(Q), mass))
        return np.stack([self.rhs(q, mass) for q in Q])

    # ------------------------------------------------------------ sweep
    def integrate(self, Q0, dt, nsteps, mass="wadg", callback=None):
        """Advance every slice of Q0 [S][3][Np][K] by nsteps LSRK steps, one
        slice after another (a serial reference)."""
        Q0 = np.asarray(Q0, dtype=np.float64)
        if Q0.ndim == 3:
            Qm = lsrk_integrate(lambda q: self.rhs_modal(q, mass), self.to_modal(Q0), dt,
                                nsteps, callback)
            return self.to_nodal(Qm)
        return np.stack([self.integrate(q, dt, nsteps, mass, callback) for q in Q0])

    # --------------------------------------------------------- diagnostics
    def energy(self, Q):
        """Weight-adjusted energy 1/2 sum_k (p^T Mt_p p + u^T Mt_u u + v^T Mt_u v)
        with Mt = Mhat M_w^{-1} Mhat, the matrix WADG uses in place of the
        weighted mass (Section 4: energy stability in the Mt-norm)."""
        Qm = self.to_modal(Q)
        Mh = self.ref.Mhat
        Mt_p = Mh[None] @ np.linalg.inv(self.Mw_p) @ Mh[None]
        Mt_u = Mh[None] @ np.linalg.inv(self.Mw_u) @ Mh[None]
        e = np.einsum("ki,kij,kj->", Qm[0], Mt_p, Qm[0])
        e += np.einsum("ki,kij,kj->", Qm[1], Mt_u, Qm[1])
        e += np.einsum("ki,kij,kj->", Qm[2], Mt_u, Qm[2])
        return 0.5 * e

    def l2_error(self, Q, exact, t, nq_err=None):
        """L2 norm over the mesh of (numerical - exact) for p, u, v together,
        by an nq_err-point tensor Gauss rule on every element (with J)."""
        N = self.N
        ref = ReferenceQuad(N, (N + 3) if nq_err is None else nq_err)
        Qm = self.to_modal(np.asarray(Q))
        xr, xs = self.cx @ ref.Vr.T, self.cx @ ref.Vs.T
        yr, ys = self.cy @ ref.Vr.T, self.cy @ ref.Vs.T
        J = xr * ys - xs * yr
        x, y = self.cx @ ref.V.T, self.cy @ ref.V.T
        ex = exact(x, y, t)
        tot = 0.0
        for f in range(3):
            d = Qm[f] @ ref.V.T - ex[f]
            tot += np.sum(ref.W[None] * J * d * d)
        return np.sqrt(tot)

    def l2_norm(self, Q, nq=None):
        """L2 norm over the mesh of a discrete state [3][Np][K] (p, u, v
        together): the square root of the integral of p^2 + u^2 + v^2 over
        every element, with the element map's Jacobian, by an nq-point tensor
        Gauss rule (default: the volume rule nq1).  The norm of the L2 errors
        of Section 5.2, applied to a difference of two discrete states."""
        ref = self.ref if nq is None or nq == self.nq1 else ReferenceQuad(self.N, nq)
        Qm = self.to_modal(np.asarray(Q, dtype=np.float64))
        xr, xs = self.cx @ ref.Vr.T, self.cx @ ref.Vs.T
        yr, ys = self.cy @ ref.Vr.T, self.cy @ ref.Vs.T
        J = xr * ys - xs * yr
        tot = 0.0
        for f in range(3):
            d = Qm[f] @ ref.V.T
            tot += np.sum(ref.W[None] * J * d * d)
        return np.sqrt(tot)

    def assemble(self, mass="wadg"):
        """Dense matrix of Q -> dQ/dt in nodal coordinates (small meshes only)."""
        n = 3 * self.Np * self.K
        L = np.zeros((n, n))
        e = np.zeros(n)
        for i in range(n):
            e[:] = 0.0
            e[i] = 1.0
            L[:, i] = self.rhs(e.reshape(3, self.Np, self.K), mass).reshape(-1)
        return L
