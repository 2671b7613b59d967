"""GPU: the three stage-kernel variants (streamed geometry, LDS-resident
geometry, split work) compute bit-identical results, on shapes that exercise the
resident kernel's work split -- several slices per pair, an odd slice count
(a pair with nothing to do in its last iteration), workgroups whose slice
range is empty, a ragged last element group -- in stage and right-hand-side
mode and in FP32; and the resident path agrees with the oracle."""

import numpy as np
import pytest

from workloads import periodic_quad_mesh, c2_layered
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


def _states(mesh, S, seed):
    return np.random.default_rng(seed).standard_normal((S, 3, mesh.Np, mesh.K))


CASES = [  # (N, nq1 - N, K1D, S, nsteps)
    (3, 2, 32, 37, 2),    # 16 groups x 16 ranges of 3 slices; ranges 13..15 empty
    (3, 2, 9, 7, 3),      # ragged second group, odd S
    (3, 1, 17, 64, 1),    # 5 groups (last ragged) x 32 ranges of 2 slices
    (2, 3, 9, 5, 2),
    (1, 1, 8, 3, 2),
]


@pytest.mark.parametrize("N,dq,K1D,S,nsteps", CASES)
def test_streamed_and_resident_bitwise(W, N, dq, K1D, S, nsteps):
    _print_case(test="kernel-paths", N=N, nq1=N + dq, K1D=K1D, S=S, nsteps=nsteps)
    mesh = periodic_quad_mesh(K1D, N, eps=0.05, warp="skew", rotate_seed=K1D)
    sol = W.Solver(mesh, nq1=N + dq, c2=c2_layered)
    Q0 = _states(mesh, S, seed=K1D + S)
    dt = 0.1 / (K1D * (N + 1) ** 2)
    out = {}
    kerns = (W.WADG_KERNEL_STREAMED, W.WADG_KERNEL_RESIDENT, W.WADG_KERNEL_SPLIT)
    for kern in kerns:
        sol.set_kernel(kern)
        assert sol.kernel_in_use() == kern
        assert sol.kernel_in_use(fp32=True) == kern
        Q = sol.upload(Q0)
        sol.integrate(Q, S, dt, nsteps)
        dQ = sol.rhs(sol.upload(Q0), S)
        Q32 = sol.upload(Q0)
        sol.integrate_fp32(Q32, S, dt, nsteps)
        out[kern] = (sol.download(Q, S), sol.download(dQ, S), sol.download(Q32, S))
    for kern in kerns[1:]:
        for a, b in zip(out[W.WADG_KERNEL_STREAMED], out[kern]):
            assert np.all(np.isfinite(a))
            assert np.array_equal(a, b), kern


def test_resident_matches_oracle_many_slices_per_pair(W):
    """32 x 32 elements, 40 slices: 16 groups x 16 ranges of 3 slices (two
    items per pair, the last of pair 1 empty); sampled slices vs oracle."""
    _print_case(test="resident-oracle", K1D=32, S=40)
    mesh = periodic_quad_mesh(32, 3, eps=0.05, warp="skew", rotate_seed=5)
    S, nsteps, dt = 40, 2, 0.1 / (32 * 16)
    Q0 = _states(mesh, S, seed=9)
    sol = W.Solver(mesh, c2=c2_layered)
    sol.set_kernel(W.WADG_KERNEL_RESIDENT)
    assert sol.kernel_in_use() == W.WADG_KERNEL_RESIDENT
    Q = sol.upload(Q0)
    sol.integrate(Q, S, dt, nsteps)
    got = sol.download(Q, S)
    o = WADGOracle(mesh, c2=c2_layered)
    for s in (0, 1, 2, 3, 38, 39):
        want = o.integrate(Q0[s:s + 1], dt, nsteps)[0]
        rel = np.linalg.norm(got[s] - want) / np.linalg.norm(want)
        assert rel < 1e-12, (s, rel)


def test_kernel_selection_rules(W):
    """AUTO: LSRK stages (FP64 and FP32) take the pipelined kernel where its
    LDS plan fits (N = 3 with nq1 <= 5 in FP64; every nq1 in FP32), else the
    split kernel; wadg_rhs the resident kernel where the geometry fits in
    LDS (N = 3 with nq1 <= 5), else the split kernel.  An explicit choice
    applies to every launch; the resident kernel is refused where the FP64
    geometry does not fit."""
    _print_case(test="kernel-selection")
    mesh = periodic_quad_mesh(4, 3, eps=0.05, warp="skew")
    s5 = W.Solver(mesh, nq1=5)
    assert s5.kernel_in_use() == W.WADG_KERNEL_PIPE
    assert s5.kernel_in_use(fp32=True) == W.WADG_KERNEL_PIPE
    assert s5.kernel_in_use(rhs=True) == W.WADG_KERNEL_RESIDENT
    for kern in (W.WADG_KERNEL_RESIDENT, W.WADG_KERNEL_STREAMED, W.WADG_KERNEL_SPLIT):
        s5.set_kernel(kern)
        assert s5.kernel_in_use() == kern
        assert s5.kernel_in_use(fp32=True) == kern
        assert s5.kernel_in_use(rhs=True) == kern
    s6 = W.Solver(mesh, nq1=6)
    assert s6.kernel_in_use() == W.WADG_KERNEL_SPLIT
    assert s6.kernel_in_use(fp32=True) == W.WADG_KERNEL_PIPE
    assert s6.kernel_in_use(rhs=True) == W.WADG_KERNEL_SPLIT
    with pytest.raises(W.WadgError) as e:
        s6.set_kernel(W.WADG_KERNEL_RESIDENT)
    assert e.value.status == W.binding.WADG_E_UNSUPPORTED


@pytest.mark.parametrize("kern", ["STREAMED", "SPLIT"])
def test_launch_order_direction_does_not_change_results(W, kern):
    """Successive stage launches walk the work items in alternating
    directions; which direction a sweep starts in depends on the context's
    launch history.  A sweep of one step (5 launches, odd) on a fresh context
    and on one whose direction was flipped by an extra right-hand side must
    agree bit for bit, in FP64 and FP32-bulk."""
    _print_case(test="launch-order", kernel=kern)
    mesh = periodic_quad_mesh(17, 3, eps=0.05, warp="skew", rotate_seed=3)
    S, dt = 9, 0.1 / (17 * 16)
    Q0 = _states(mesh, S, seed=21)
    outs = []
    for flip in (0, 1):
        sol = W.Solver(mesh, c2=c2_layered)
        sol.set_kernel(getattr(W, "WADG_KERNEL_" + kern))
        if flip:
            sol.rhs(sol.upload(Q0), S)
        Q = sol.upload(Q0)
        sol.integrate(Q, S, dt, 1)
        Q32 = sol.upload(Q0)
        sol.integrate_fp32(Q32, S, dt, 1)
        outs.append((sol.download(Q, S), sol.download(Q32, S)))
    for a, b in zip(outs[0], outs[1]):
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b)
