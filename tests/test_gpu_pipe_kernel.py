"""GPU: the persistent pipelined stage kernel (WADG_KERNEL_PIPE) against the
split kernel (bitwise: same arithmetic in the same order) and against the
oracle, on shapes that exercise its slice runs -- one run per group and
several, runs of one slice (no prefetch), more runs than slices, a ragged
last element group, N = 1..3 with quadratures that fit -- in FP64 and
FP32-bulk; at full size in the benchmark's launch configuration (its
non-temporal instances), every output value against the split kernel's;
and its selection rules."""

import numpy as np
import pytest

from workloads import periodic_quad_mesh, c2_layered, make_problem
from oracle import WADGOracle

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


CASES = [  # (N, nq1 - N, K1D, S, nsteps)
    (3, 2, 32, 37, 2),    # 16 groups x 16 runs: runs of 2 and 3 slices
    (3, 2, 9, 7, 3),      # 2 groups (ragged second) x 7 runs of one slice
    (3, 2, 128, 3, 1),    # 256 groups x 1 run of 3 slices
    (3, 1, 17, 64, 1),    # 5 groups (last ragged) x 51 runs
    (2, 2, 9, 6, 2),
    (2, 3, 9, 5, 2),
    (1, 1, 8, 3, 2),
    (1, 2, 24, 300, 1),   # 9 groups x 28 runs of 10-11 slices
]


@pytest.mark.parametrize("N,dq,K1D,S,nsteps", CASES)
def test_pipe_equals_split_bitwise(W, N, dq, K1D, S, nsteps):
    _print_case(test="pipe-vs-split", N=N, nq1=N + dq, K1D=K1D, S=S, nsteps=nsteps)
    mesh = periodic_quad_mesh(K1D, N, eps=0.05, warp="skew", rotate_seed=K1D)
    sol = W.Solver(mesh, nq1=N + dq, c2=c2_layered)
    sol.set_c2_scale(1.3)                    # the pressure weights carry the scale
    Q0 = np.random.default_rng(K1D + S).standard_normal((S, 3, mesh.Np, mesh.K))
    dt = 0.1 / (K1D * (N + 1) ** 2)
    out = {}
    for kern in (W.WADG_KERNEL_SPLIT, W.WADG_KERNEL_PIPE):
        sol.set_kernel(kern)
        assert sol.kernel_in_use() == kern
        assert sol.kernel_in_use(fp32=True) == kern
        Q = sol.upload(Q0)
        sol.integrate(Q, S, dt, nsteps)
        Q32 = sol.upload(Q0)
        sol.integrate_fp32(Q32, S, dt, nsteps)
        out[kern] = (sol.download(Q, S), sol.download(Q32, S))
    for a, b in zip(out[W.WADG_KERNEL_SPLIT], out[W.WADG_KERNEL_PIPE]):
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b)


def test_pipe_full_size_equals_split_bitwise(W):
    """wadg128 at full size (256 slices x 10 steps, heterogeneous c^2) as the
    benchmark runs it: the automatic choice takes the pipelined kernel's
    non-temporal instances, since a launch's state far exceeds the caches.
    Every output value, FP64 and FP32-bulk, equals the split kernel's."""
    import torch
    _print_case(test="pipe-vs-split-full-size", workload="wadg128")
    prob = make_problem("wadg128")
    sol = W.Solver.from_problem(prob)
    assert sol.kernel_in_use() == W.WADG_KERNEL_PIPE
    assert sol.kernel_in_use(fp32=True) == W.WADG_KERNEL_PIPE
    out = {}
    for kern in (W.WADG_KERNEL_AUTO, W.WADG_KERNEL_SPLIT):
        sol.set_kernel(kern)
        Q = sol.upload(prob.Q0)
        sol.integrate(Q, prob.S, prob.dt, prob.nsteps)
        Q32 = sol.upload(prob.Q0)
        sol.integrate_fp32(Q32, prob.S, prob.dt, prob.nsteps)
        torch.cuda.synchronize()
        out[kern] = (Q, Q32)
    for a, b in zip(out[W.WADG_KERNEL_AUTO], out[W.WADG_KERNEL_SPLIT]):
        assert bool(torch.isfinite(a).all())
        assert torch.equal(a, b)


def test_pipe_matches_oracle(W):
    """40 slices of a 24 x 24 mesh (9 groups, ragged last): every slice run
    holds several slices; sampled slices against the oracle at 1e-12, element
    by element."""
    _print_case(test="pipe-oracle", K1D=24, S=40)
    mesh = periodic_quad_mesh(24, 3, eps=0.05, warp="skew", rotate_seed=2)
    S, nsteps, dt = 40, 2, 0.1 / (24 * 16)
    Q0 = np.random.default_rng(5).standard_normal((S, 3, mesh.Np, mesh.K))
    sol = W.Solver(mesh, c2=c2_layered)
    sol.set_kernel(W.WADG_KERNEL_PIPE)
    Q = sol.upload(Q0)
    sol.integrate(Q, S, dt, nsteps)
    got = sol.download(Q, S)
    o = WADGOracle(mesh, c2=c2_layered)
    for s in (0, 1, 13, 27, 38, 39):
        want = o.integrate(Q0[s:s + 1], dt, nsteps)[0]
        assert np.linalg.norm(got[s] - want) <= 1e-12 * np.linalg.norm(want), s
        assert np.max(np.abs(got[s] - want)) <= 1e-12 * np.max(np.abs(want)), s


def test_pipe_selection_rules(W):
    """PIPE applies to LSRK stages of two or more slices; right-hand sides
    and one-slice sweeps take the split kernel; PIPE is refused where its
    FP64 tiles, metric planes and weights do not fit in LDS (N = 4, and
    N = 3 with six quadrature points per direction)."""
    _print_case(test="pipe-selection")
    mesh = periodic_quad_mesh(4, 3, eps=0.05, warp="skew")
    s = W.Solver(mesh)
    s.set_kernel(W.WADG_KERNEL_PIPE)
    assert s.kernel_in_use() == W.WADG_KERNEL_PIPE
    assert s.kernel_in_use(fp32=True) == W.WADG_KERNEL_PIPE
    assert s.kernel_in_use(rhs=True) == W.WADG_KERNEL_SPLIT
    Q0 = np.random.default_rng(1).standard_normal((1, 3, mesh.Np, mesh.K))
    a, b = s.upload(Q0), s.upload(Q0)
    s.integrate(a, 1, 1e-3, 2)                 # one slice: the split kernel
    s.set_kernel(W.WADG_KERNEL_SPLIT)
    s.integrate(b, 1, 1e-3, 2)
    assert np.array_equal(s.download(a, 1), s.download(b, 1))
    for N, nq1 in ((4, 6), (3, 6)):
        m = periodic_quad_mesh(4, N, eps=0.05, warp="skew")
        sn = W.Solver(m, nq1=nq1)
        with pytest.raises(W.WadgError) as e:
            sn.set_kernel(W.WADG_KERNEL_PIPE)
        assert e.value.status == W.binding.WADG_E_UNSUPPORTED
