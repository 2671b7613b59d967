"""Convenience layer over the C ABI: device memory and streams from torch,
layout conversion on the host.  All arithmetic of the sweep runs in the HIP
library."""

import numpy as np

from . import binding as B


class Solver:
    """One WADG context on one HIP device.

    ``mesh`` is any object with ``N, x, y, etoe, etof`` (GLL node coordinates
    [K][(N+1)^2], connectivity [K][4]); ``c2`` an optional callable
    ``c2(x, y)`` evaluated at the volume quadrature points, or ``c2q`` the
    values there, [K][nq1^2] (at most one of the two).
    """

    def __init__(self, mesh, nq1=None, c2=None, tau_p=1.0, tau_u=1.0, device=0, c2q=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        N = int(mesh.N)
        nq1 = N + 2 if nq1 is None else int(nq1)
        if c2 is not None and c2q is not None:
            raise ValueError("give c2 or c2q, not both")
        desc = B.MeshDesc(N, nq1, mesh.x, mesh.y, mesh.etoe, mesh.etof,
                          None if c2q is None else np.asarray(c2q, dtype=np.float64),
                          tau_p, tau_u)
        if c2 is not None:
            xq, yq = B.wadg_quadrature_points(desc)
            desc = B.MeshDesc(N, nq1, mesh.x, mesh.y, mesh.etoe, mesh.etof,
                              np.asarray(c2(xq, yq), dtype=np.float64), tau_p, tau_u)
        self.desc = desc
        self.N, self.nq1, self.K = N, nq1, desc.K
        self.Np = (N + 1) ** 2
        with torch.cuda.device(self.device):
            self.ctx = B.wadg_create(desc, device)
        self.slice_doubles = B.wadg_state_doubles(self.ctx)

    @classmethod
    def from_problem(cls, prob, device=0):
        return cls(prob.mesh, nq1=prob.nq1, c2=prob.c2, tau_p=prob.tau_p, tau_u=prob.tau_u,
                   device=device)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            B.wadg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- memory ----------------------------------------------------------
    def empty_state(self, S):
        return self.torch.zeros(S * self.slice_doubles, dtype=self.torch.float64,
                                device=self.device)

    def workspace(self, S):
        n = B.wadg_workspace_bytes(self.ctx, S) // 8
        return self.torch.empty(n, dtype=self.torch.float64, device=self.device)

    def upload(self, Qn):
        """Natural [S][3][Np][K] host array -> tiled device tensor."""
        t = B.tile_state(np.asarray(Qn).reshape(-1, 3, self.Np, self.K))
        return self.torch.from_numpy(t.reshape(-1)).to(self.device)

    def download(self, Q, S):
        """Tiled device tensor -> natural [S][3][Np][K] host array."""
        G = self.slice_doubles // (3 * self.Np * B.TILE_LANES)
        h = Q.detach().cpu().numpy().reshape(S, G, 3, self.Np, B.TILE_LANES)
        return B.untile_state(h, self.K)

    # -- the sweep -------------------------------------------------------
    def rhs(self, Q, S, out=None, stream=None):
        out = self.empty_state(S) if out is None else out
        B.wadg_rhs(self.ctx, Q, out, S, stream)
        return out

    def integrate(self, Q, S, dt, nsteps, work=None, stream=None):
        work = self.workspace(S) if work is None else work
        B.wadg_integrate(self.ctx, Q, work, S, dt, nsteps, stream)
        return Q

    def workspace_fp32(self, S):
        n = B.wadg_workspace_bytes_fp32(self.ctx, S) // 4
        return self.torch.empty(n, dtype=self.torch.float32, device=self.device)

    def integrate_fp32(self, Q, S, dt, nsteps, work=None, stream=None):
        """FP32-bulk sweep: FP64 Q in and out, FP32 interior."""
        work = self.workspace_fp32(S) if work is None else work
        B.wadg_integrate_fp32(self.ctx, Q, work, S, dt, nsteps, stream)
        return Q

    def parareal(self, y0, S, dt, nsteps_fine, nsteps_coarse, max_iter, tol, fine_fp32=False,
                 U=None, work=None, stream=None):
        """Parareal over S slices from the device state y0 (one slice).
        Returns (U device tensor of S+1 slices, iterations, last change)."""
        U = self.empty_state(S + 1) if U is None else U
        if work is None:
            n = B.wadg_parareal_workspace_bytes(self.ctx, S, fine_fp32) // 8 + 1
            work = self.torch.empty(n, dtype=self.torch.float64, device=self.device)
        it, ch = B.wadg_parareal(self.ctx, y0, U, work, S, dt, nsteps_fine, nsteps_coarse,
                                 max_iter, tol, fine_fp32, stream)
        return U, it, ch

    def scratch(self, nbytes):
        """Device scratch of at least nbytes for the reductions, kept by the
        solver and grown when a call needs more (torch device memory)."""
        have = getattr(self, "_scratch", None)
        if have is None or have.numel() * 8 < nbytes:
            self._scratch = self.torch.empty(max(1, -(-nbytes // 8)), dtype=self.torch.float64,
                                             device=self.device)
        return self._scratch

    def norms(self, A, Bt=None, S=1, stream=None, check_finite=True):
        sc = self.scratch(B.wadg_norms_workspace_bytes(self.ctx, S))
        return B.wadg_norms(self.ctx, A, Bt, S, sc, stream, check_finite=check_finite)

    def l2_norms(self, A, Bt=None, S=1, stream=None, check_finite=True):
        """Per slice (||A - Bt||_L2, ||Bt||_L2) with the element Jacobians."""
        sc = self.scratch(B.wadg_l2_norms_workspace_bytes(self.ctx, S))
        return B.wadg_l2_norms(self.ctx, A, Bt, S, sc, stream, check_finite=check_finite)

    def set_schedule(self, groups_per_tile, slices_per_tile=0):
        B.wadg_set_schedule(self.ctx, groups_per_tile, slices_per_tile)

    def set_kernel(self, kernel):
        """WADG_KERNEL_AUTO, _STREAMED, _RESIDENT, _SPLIT or _PIPE (see wadg_set_kernel)."""
        B.wadg_set_kernel(self.ctx, kernel)

    def kernel_in_use(self, rhs=False, fp32=False):
        return B.wadg_kernel_in_use(self.ctx, rhs, fp32)

    # -- sensitivities ---------------------------------------------------
    def set_c2_scale(self, gamma):
        """Use c^2 = gamma * c2 (the wave speed given at construction)."""
        B.wadg_set_c2_scale(self.ctx, gamma)
        self.c2_scale = float(gamma)

    c2_scale = 1.0      # the context's current scale (the library's default)

    def adjoint_workspace(self, nsteps):
        n = B.wadg_adjoint_workspace_bytes(self.ctx, nsteps) // 8 + 1
        return self.torch.empty(n, dtype=self.torch.float64, device=self.device)

    def forward_checkpoints(self, y0, S, dt, nsteps, work=None, stream=None):
        """One trajectory from the device state y0 (one slice) over S slices of
        nsteps steps; returns the S+1 slice-boundary states (device tensor)."""
        chk = self.empty_state(S + 1)
        chk[: self.slice_doubles].copy_(y0.reshape(-1)[: self.slice_doubles])
        work = self.adjoint_workspace(nsteps) if work is None else work
        B.wadg_forward_checkpoints(self.ctx, chk, work, S, dt, nsteps, stream)
        return chk

    def adjoint(self, chk, seed, S, dt, nsteps, work=None, stream=None):
        """Reverse sweep: (dJ/dq(0) device tensor, gamma dJ/dgamma) for
        seed = dJ/dq(T) and the checkpoints of ``forward_checkpoints``."""
        grad = self.empty_state(1)
        work = self.adjoint_workspace(nsteps) if work is None else work
        d = B.wadg_adjoint(self.ctx, chk, seed.contiguous(), grad, work, S, dt, nsteps, stream)
        return grad, d


class Batch:
    """Many independent problems (same degree and quadrature) advanced
    together through the batch C ABI.

    ``meshes``: list of meshes (as for ``Solver``); ``S``: slices per
    problem; ``c2``: optional callable evaluated at each mesh's volume
    quadrature points.
    """

    def __init__(self, meshes, S, nq1=None, c2=None, tau_p=1.0, tau_u=1.0, device=0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        N = int(meshes[0].N)
        nq1 = N + 2 if nq1 is None else int(nq1)
        descs = []
        for m in meshes:
            d = B.MeshDesc(N, nq1, m.x, m.y, m.etoe, m.etof, None, tau_p, tau_u)
            if c2 is not None:
                xq, yq = B.wadg_quadrature_points(d)
                d = B.MeshDesc(N, nq1, m.x, m.y, m.etoe, m.etof,
                               np.asarray(c2(xq, yq), dtype=np.float64), tau_p, tau_u)
            descs.append(d)
        self.N, self.nq1, self.Np = N, nq1, (N + 1) ** 2
        self.S = [int(s) for s in S]
        self.K = [d.K for d in descs]
        with torch.cuda.device(self.device):
            self.b = B.wadg_batch_create(descs, self.S, device)
        self.offset, self.pack = B.wadg_batch_layout(self.b, len(descs))
        self.total = int(self.offset[-1])

    def close(self):
        if getattr(self, "b", None) is not None:
            B.wadg_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self):
        n = B.wadg_batch_workspace_bytes(self.b) // 8
        return self.torch.empty(n, dtype=self.torch.float64, device=self.device)

    def upload(self, Q0):
        """Q0: list of natural [S_i][3][Np][K_i] host arrays -> batch state."""
        h = np.zeros(self.total)
        for i, q in enumerate(Q0):
            h[self.offset[i]:self.offset[i + 1]] = B.pack_batch_problem(q, self.pack[i])
        return self.torch.from_numpy(h).to(self.device)

    def download(self, Q, which=None):
        h = Q.detach().cpu().numpy()
        idx = range(len(self.S)) if which is None else which
        return [B.unpack_batch_problem(h[self.offset[i]:self.offset[i + 1]], self.S[i], self.K[i],
                                       self.Np, self.pack[i]) for i in idx]

    def integrate(self, Q, dt, nsteps, work=None, stream=None):
        work = self.workspace() if work is None else work
        B.wadg_batch_integrate(self.b, Q, work, dt, nsteps, stream)
        return Q

    def set_schedule(self, wg_per_cu, order=0):
        B.wadg_batch_set_schedule(self.b, wg_per_cu, order)

    def set_runs(self, run_slices):
        """Pipelined kernel with runs of at most run_slices slices per
        workgroup (0: the item schedule of set_schedule)."""
        B.wadg_batch_set_runs(self.b, run_slices)

    def tune(self, Q, dt, work=None, reps=3, stream=None):
        work = self.workspace() if work is None else work
        return B.wadg_batch_tune(self.b, Q, work, dt, reps, stream)

    def capture(self, Q, work, dt, nsteps):
        B.wadg_batch_capture(self.b, Q, work, dt, nsteps)

    def replay(self, stream=None):
        B.wadg_batch_replay(self.b, stream)

    def release_graph(self):
        B.wadg_batch_release_graph(self.b)
