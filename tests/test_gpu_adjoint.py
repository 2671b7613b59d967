"""GPU: the discrete adjoint of the sweep (the library's reverse LSRK sweep
with the transposed operator, recomputing each slice from its checkpoint).

* oracle-sized (adj4): checkpointed forward vs the oracle stepper, gradient
  with respect to the start state and the c^2 scale vs the oracle's
  terminal-objective gradient (dense transposition, tangent-linear);
* the torch autograd function: gradients vs central finite differences of
  the GPU forward sweep;
* full size (adj128: 128 x 128 elements, 128 checkpointed slices of 10
  steps): central finite differences on gamma and on three seeded unit
  directions of the start state, and the dot-product identity
  <Phi x, w> = <x, Phi^T w> of the forward and adjoint sweeps.

Tolerances: gradients against the oracle 1e-12 relative in the l2 norm and
element by element (max |difference| <= 1e-12 max |oracle|), dJ/dgamma 1e-12
relative (both sides FP64; the measured errors are near 1e-14); finite
differences as derived in the tests.
"""

import numpy as np
import pytest

from workloads import make_sensitivity_problem
from oracle import TerminalObjective, WADGOracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1608_03836_amd as pkg
    return pkg


def _print_case(**kw):
    print("CASE", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _solver(W, prob):
    sol = W.Solver(prob.mesh, nq1=prob.nq1, c2=prob.c0, tau_p=prob.tau_p, tau_u=prob.tau_u)
    sol.set_c2_scale(prob.gamma)
    return sol


def _seed(sol, qT_nat, p_target):
    g = np.zeros_like(qT_nat)
    g[0] = 2.0 * (qT_nat[0] - p_target)
    return sol.upload(g[None])


def _assert_gradient(g_gpu, g_orc, dg_gpu, dg_orc, tol=1e-12):
    """The FP64 bar, element by element: relative l2 error and max |error|
    over max |oracle| of the start-state gradient, relative error of
    dJ/dgamma."""
    assert np.linalg.norm(g_gpu - g_orc) <= tol * np.linalg.norm(g_orc)
    assert np.max(np.abs(g_gpu - g_orc)) <= tol * np.max(np.abs(g_orc))
    assert abs(dg_gpu - dg_orc) <= tol * abs(dg_orc), (dg_gpu, dg_orc)


def test_adjoint_matches_oracle(W):
    _print_case(test="adjoint-oracle", workload="adj4")
    prob = make_sensitivity_problem("adj4")
    sol = _solver(W, prob)
    y0 = sol.upload(prob.y0[None])
    chk = sol.forward_checkpoints(y0, prob.S, prob.dt, prob.nsteps)
    states = sol.download(chk, prob.S + 1)
    o = WADGOracle(prob.mesh, c2=lambda x, y: prob.gamma * prob.c0(x, y))
    want = prob.y0
    for s in range(prob.S):
        want = o.integrate(want, prob.dt, prob.nsteps)
        rel = np.linalg.norm(states[s + 1] - want) / np.linalg.norm(want)
        assert rel <= 1e-12, (s, rel)
    seed = _seed(sol, states[-1], prob.p_target)
    grad, dscale = sol.adjoint(chk, seed, prob.S, prob.dt, prob.nsteps)
    g_gpu = sol.download(grad, 1)[0]
    obj = TerminalObjective(prob.mesh, c0=prob.c0)
    J, g_orc, dgamma = obj.gradient(prob.y0, prob.p_target, prob.gamma, prob.dt,
                                    prob.S * prob.nsteps)
    rel = np.linalg.norm(g_gpu - g_orc) / np.linalg.norm(g_orc)
    mx = np.max(np.abs(g_gpu - g_orc)) / np.max(np.abs(g_orc))
    print(f"adj4: |grad - oracle|/|oracle| = {rel:.3e}, max {mx:.3e}; dJ/dgamma gpu "
          f"{dscale / prob.gamma:.15e} oracle {dgamma:.15e}", flush=True)
    _assert_gradient(g_gpu, g_orc, dscale / prob.gamma, dgamma)


@pytest.mark.parametrize("N", [1, 2, 4])
def test_adjoint_other_degrees_match_oracle(W, N):
    """The adjoint sweep of other degrees (the adjoint mass kernel and the
    apply-A launches of degree N) against the oracle's terminal-objective
    gradient, on 4 x 4 elements."""
    _print_case(test="adjoint-degrees", N=N)
    prob = make_sensitivity_problem("adj4", N=N)
    sol = _solver(W, prob)
    y0 = sol.upload(prob.y0[None])
    chk = sol.forward_checkpoints(y0, prob.S, prob.dt, prob.nsteps)
    states = sol.download(chk, prob.S + 1)
    seed = _seed(sol, states[-1], prob.p_target)
    grad, dscale = sol.adjoint(chk, seed, prob.S, prob.dt, prob.nsteps)
    g_gpu = sol.download(grad, 1)[0]
    obj = TerminalObjective(prob.mesh, c0=prob.c0)
    J, g_orc, dgamma = obj.gradient(prob.y0, prob.p_target, prob.gamma, prob.dt,
                                    prob.S * prob.nsteps)
    rel = np.linalg.norm(g_gpu - g_orc) / np.linalg.norm(g_orc)
    print(f"adj4 N={N}: |grad - oracle|/|oracle| = {rel:.3e}", flush=True)
    _assert_gradient(g_gpu, g_orc, dscale / prob.gamma, dgamma)


def test_autograd_function_matches_finite_differences(W):
    import torch
    from paper_1608_03836_amd.autograd import sweep, pressure_mask
    _print_case(test="adjoint-autograd", workload="adj4-K1D8")
    prob = make_sensitivity_problem("adj4", K1D=8)
    sol = _solver(W, prob)
    mask = pressure_mask(sol)
    target = sol.upload(np.stack([prob.p_target, np.zeros_like(prob.p_target),
                                  np.zeros_like(prob.p_target)])[None])

    def J_of(y0, gamma):
        qT = sweep(sol, y0, gamma, prob.S, prob.dt, prob.nsteps)
        return torch.sum((mask * (qT - target)) ** 2)

    y0 = sol.upload(prob.y0[None]).requires_grad_(True)
    plain = sol.upload(prob.y0[None])
    sol.integrate(plain, 1, prob.dt, 3)
    gamma = torch.tensor(prob.gamma, dtype=torch.float64, requires_grad=True)
    J = J_of(y0 * 1.0, gamma * 1.1)
    J.backward()
    # the differentiable sweep leaves the solver's c^2 scale as it found it
    assert sol.c2_scale == prob.gamma
    again = sol.upload(prob.y0[None])
    sol.integrate(again, 1, prob.dt, 3)
    assert torch.equal(plain, again)
    y0.grad = None
    gamma.grad = None
    J = J_of(y0, gamma)
    J.backward()
    with torch.no_grad():
        h = 1e-6
        fd = (J_of(y0, gamma + h) - J_of(y0, gamma - h)).item() / (2 * h)
        assert abs(fd - gamma.grad.item()) <= 1e-6 * abs(fd), (fd, gamma.grad.item())
        rng = np.random.default_rng(3)
        for _ in range(3):
            d = rng.standard_normal(prob.y0.shape)
            d /= np.linalg.norm(d)
            dt_ = sol.upload(d[None])
            hd = 1e-3   # J is quadratic in y0: central differences exact up to rounding
            fd = (J_of(y0 + hd * dt_, gamma) - J_of(y0 - hd * dt_, gamma)).item() / (2 * hd)
            an = torch.sum(y0.grad * dt_).item()
            assert abs(fd - an) <= 1e-9 * J.item(), (fd, an)



def test_autograd_drops_the_gradient_of_padding_lanes(W):
    """On a ragged mesh (81 elements, 47 padding lanes in the last group) a
    loss that also depends on the output's padding lanes gives the same
    gradients, bit for bit, as the loss over real elements only: padding
    holds no state, so its gradient is dropped, and the returned gradient is
    zero there."""
    import torch
    from paper_1608_03836_amd.autograd import sweep, element_mask
    _print_case(test="adjoint-autograd-padding", workload="adj4-K1D9")
    prob = make_sensitivity_problem("adj4", K1D=9)
    sol = _solver(W, prob)
    assert sol.K % 64 != 0
    em = element_mask(sol)
    grads = []
    for with_padding in (False, True):
        y0 = sol.upload(prob.y0[None]).requires_grad_(True)
        gamma = torch.tensor(prob.gamma, dtype=torch.float64, requires_grad=True)
        qT = sweep(sol, y0, gamma, prob.S, prob.dt, prob.nsteps)
        J = torch.sum((em * qT) ** 2)
        if with_padding:
            J = J + 5.0 * torch.sum((1.0 - em) * qT)
        J.backward()
        grads.append((y0.grad.clone(), gamma.grad.clone()))
    assert torch.equal(grads[0][0], grads[1][0]) and torch.equal(grads[0][1], grads[1][1])
    assert torch.all(grads[1][0][em == 0] == 0) and torch.any(grads[1][0] != 0)


def test_full_size_adjoint_fd_and_transpose(W):
    import torch
    _print_case(test="adjoint-full", workload="adj128")
    prob = make_sensitivity_problem("adj128")
    sol = _solver(W, prob)
    n1 = sol.slice_doubles
    y0 = sol.upload(prob.y0[None])
    work = sol.adjoint_workspace(prob.nsteps)
    target = np.zeros((1, 3) + prob.p_target.shape)
    target[0, 0] = prob.p_target
    target = sol.upload(target)
    from paper_1608_03836_amd.autograd import pressure_mask
    mask = pressure_mask(sol)

    def forward(y, gamma):
        sol.set_c2_scale(gamma)
        chk = sol.forward_checkpoints(y, prob.S, prob.dt, prob.nsteps, work=work)
        return chk, chk[prob.S * n1:]

    def J_of(y, gamma):
        _, qT = forward(y, gamma)
        return torch.sum((mask * (qT - target)) ** 2).item()

    chk, qT = forward(y0, prob.gamma)
    J = torch.sum((mask * (qT - target)) ** 2).item()
    seed = (2.0 * mask * (qT - target)).contiguous()
    grad, dscale = sol.adjoint(chk, seed, prob.S, prob.dt, prob.nsteps, work=work)
    h = 1e-6
    fd = (J_of(y0, prob.gamma + h) - J_of(y0, prob.gamma - h)) / (2 * h)
    print(f"adj128: J = {J:.6e}, dJ/dgamma adjoint {dscale:.10e} fd {fd:.10e}", flush=True)
    assert abs(fd - dscale / prob.gamma) <= 1e-5 * abs(fd)
    rng = np.random.default_rng(5)
    for i in range(3):
        d = rng.standard_normal(prob.y0.shape)
        d /= np.linalg.norm(d)
        dd = sol.upload(d[None])
        hd = 1e-3
        fd = (J_of(y0 + hd * dd, prob.gamma) - J_of(y0 - hd * dd, prob.gamma)) / (2 * hd)
        an = torch.sum(grad * dd).item()
        print(f"adj128: direction {i}: adjoint {an:.10e} fd {fd:.10e}", flush=True)
        assert abs(fd - an) <= 1e-9 * J
    # <Phi x, w> = <x, Phi^T w>: the adjoint of a seed w is Phi^T w
    x = sol.upload(rng.standard_normal(prob.y0.shape)[None])
    w = sol.upload(rng.standard_normal(prob.y0.shape)[None])
    _, Phix = forward(x, prob.gamma)
    chk, _ = forward(y0, prob.gamma)
    PhiTw, _ = sol.adjoint(chk, w, prob.S, prob.dt, prob.nsteps, work=work)
    lhs = torch.sum(Phix * w).item()
    rhs = torch.sum(x * PhiTw).item()
    print(f"adj128: <Phi x, w> = {lhs:.15e}, <x, Phi^T w> = {rhs:.15e}", flush=True)
    assert abs(lhs - rhs) <= 1e-12 * torch.linalg.norm(x).item() * torch.linalg.norm(w).item()


def test_adjoint_kernel_variants_bitwise(W):
    """The adjoint's apply-A launches run on the split kernel (default) or
    the streamed kernel; forward checkpoints and the reverse sweep give the
    same bits either way."""
    _print_case(test="adjoint-kernels", workload="adj4-K1D8")
    prob = make_sensitivity_problem("adj4", K1D=8)
    outs = []
    for kern in (W.WADG_KERNEL_AUTO, W.WADG_KERNEL_STREAMED):
        sol = _solver(W, prob)
        sol.set_kernel(kern)
        y0 = sol.upload(prob.y0[None])
        chk = sol.forward_checkpoints(y0, prob.S, prob.dt, prob.nsteps)
        states = sol.download(chk, prob.S + 1)
        seed = _seed(sol, states[-1], prob.p_target)
        grad, dscale = sol.adjoint(chk, seed, prob.S, prob.dt, prob.nsteps)
        outs.append((states, sol.download(grad, 1)[0], dscale))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.all(np.isfinite(outs[0][1]))
    assert np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]


def test_adjoint_on_a_caller_stream_is_bitwise_the_same(W):
    """The reverse sweep orders its recompute stream against the caller's
    stream with events; run on a non-default torch stream (the binding
    passes torch's current stream), the gradient and the c^2 sensitivity
    equal the default-stream run bit for bit."""
    import contextlib
    import torch
    _print_case(test="adjoint-stream", workload="adj4-K1D8")
    prob = make_sensitivity_problem("adj4", K1D=8, S=5)
    outs = []
    for side in (None, torch.cuda.Stream()):
        sol = _solver(W, prob)
        with (torch.cuda.stream(side) if side is not None else contextlib.nullcontext()):
            y0 = sol.upload(prob.y0[None])
            chk = sol.forward_checkpoints(y0, prob.S, prob.dt, prob.nsteps)
            seed = (2.0 * chk[prob.S * sol.slice_doubles:]).contiguous()
            grad, dscale = sol.adjoint(chk, seed, prob.S, prob.dt, prob.nsteps)
            g = sol.download(grad, 1)[0]
        torch.cuda.synchronize()
        outs.append((g, dscale))
    assert np.all(np.isfinite(outs[0][0]))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]
