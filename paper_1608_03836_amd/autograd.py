"""Differentiable WADG sweep for torch: the forward pass runs the HIP
sweep with checkpoints at slice boundaries, the backward pass the library's
discrete adjoint (the reverse sweep of the LSRK recursion with the
transposed operator, recomputing each slice from its checkpoint).

    qT = sweep(solver, y0, gamma, S, dt, nsteps)

advances the start state y0 (one slice of the tiled state layout, a float64
device tensor) over S slices of nsteps steps with c^2 = gamma * c2, and is
differentiable with respect to y0 and gamma (a 0-d float64 tensor).
"""

import torch


class WadgSweep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y0, gamma, solver, S, dt, nsteps):
        g = float(gamma)
        with _scaled(solver, g):
            chk = solver.forward_checkpoints(y0.detach(), S, dt, nsteps)
        ctx.solver, ctx.S, ctx.dt, ctx.nsteps, ctx.gamma = solver, S, dt, nsteps, g
        ctx.save_for_backward(chk)
        n1 = solver.slice_doubles
        return chk[S * n1:(S + 1) * n1].clone()

    @staticmethod
    def backward(ctx, grad_qT):
        (chk,) = ctx.saved_tensors
        solver = ctx.solver
        # padding lanes of the tiled layout hold no state: their gradient is
        # dropped (the adjoint requires a seed that is zero there), and the
        # returned gradient is zero there
        mask = element_mask(solver)
        seed = grad_qT.detach().reshape(-1) * mask
        with _scaled(solver, ctx.gamma):
            grad_y0, d_scale = solver.adjoint(chk, seed, ctx.S, ctx.dt, ctx.nsteps)
        grad_gamma = torch.tensor(d_scale / ctx.gamma, dtype=torch.float64,
                                  device=grad_qT.device)
        return grad_y0 * mask, grad_gamma, None, None, None, None


class _scaled:
    """Run with c^2 = gamma * c2 on the solver, then restore the scale it had
    before, so that a differentiable sweep leaves the solver's later plain
    calls as they were."""

    def __init__(self, solver, gamma):
        self.solver, self.gamma = solver, gamma

    def __enter__(self):
        self.prev = self.solver.c2_scale
        self.solver.set_c2_scale(self.gamma)

    def __exit__(self, *exc):
        self.solver.set_c2_scale(self.prev)
        return False


def sweep(solver, y0, gamma, S, dt, nsteps):
    return WadgSweep.apply(y0, gamma, solver, S, dt, nsteps)


def element_mask(solver):
    """1.0 on every entry of real elements in one slice of the tiled layout,
    0.0 on the padding lanes of the last element group."""
    G = solver.slice_doubles // (3 * solver.Np * 64)
    k = torch.arange(G * 64).reshape(G, 1, 1, 64)
    m = (k < solver.K).to(torch.float64).expand(G, 3, solver.Np, 64)
    return m.reshape(-1).to(solver.device)


def pressure_mask(solver):
    """1.0 on the pressure entries of real elements in one slice of the tiled
    layout, 0.0 elsewhere (velocity entries and padding lanes)."""
    G = solver.slice_doubles // (3 * solver.Np * 64)
    m = torch.zeros(G, 3, solver.Np, 64, dtype=torch.float64)
    k = torch.arange(G * 64).reshape(G, 64)
    m[:, 0, :, :] = (k < solver.K).to(torch.float64)[:, None, :]
    return m.reshape(-1).to(solver.device)
