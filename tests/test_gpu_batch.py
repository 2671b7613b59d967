"""GPU: batches of independent problems (the batch C ABI) -- every problem
of a batch advanced by one launch per LSRK stage equals the same problem
advanced alone (bitwise: the same per-item arithmetic) and the oracle (to
the FP64 bar); results are bitwise independent of the schedule and of the
autotuner's choice; a captured HIP graph replays the eager sweep exactly,
replay after replay, with eager work and synchronisations between them, and
a recapture or release waits for replays still queued; and the full
1000-problem workload matches the single-problem path on sampled problems."""

import numpy as np
import pytest

from workloads import make_batch
from oracle import WADGOracle

pytestmark = pytest.mark.gpu

# indices into the 1000-problem batch: meshes of 4, 16 and 25 elements packed
# into one lane group per virtual slice, of 36, 49, 144, 169, 196 and 225
# packed over several groups, and one of 121 elements unpacked (several
# groups, one slice each)
MEMBERS = [3, 5, 2, 0, 1, 4, 6, 8, 10, 11, 12]


@pytest.fixture(scope="module")
def W():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1608_03836_amd as pkg
    return pkg


def _print_case(**kw):
    print("CASE", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


@pytest.fixture(scope="module")
def small(W):
    probs = make_batch(members=MEMBERS)
    batch = W.Batch([p.mesh for p in probs], [p.S for p in probs])
    return probs, batch


def test_members_cover_packed_and_multi_group(small):
    probs, batch = small
    Ks = sorted(p.mesh.K for p in probs)
    assert Ks[0] <= 16 and Ks[-1] > 128
    assert max(batch.pack) > 1 and min(batch.pack) == 1
    Ps = [(p.mesh.K, P) for p, P in zip(probs, batch.pack)]
    assert any(P > 1 and P * K <= 64 for K, P in Ps)
    assert any(P > 1 and P * K > 64 for K, P in Ps)
    assert any(P == 1 and K > 64 for K, P in Ps)
    # the documented rule: P in [1, min(S, 64)] moving the fewest bytes per
    # stage (state tiles per item + geometry per virtual group), smallest P
    Np, nq = 16, 5
    state_item = 4 * 3 * Np * 64 * 8
    geo_group = ((6 * nq * nq + 12 * nq) * 8 + 8 * 4) * 64
    for p, P in zip(probs, batch.pack):
        K, S = p.mesh.K, p.S
        cost = {Q: (-(-S // Q)) * (-(-(Q * K) // 64)) * state_item + (-(-(Q * K) // 64)) * geo_group
                for Q in range(1, min(S, 64) + 1)}
        assert P == min(cost, key=lambda Q: (cost[Q], Q)), (K, S, P)


def test_batch_equals_single_problem_path(W, small):
    _print_case(test="batch-vs-single", problems=len(small[0]))
    probs, batch = small
    dts = [p.dt for p in probs]
    Q = batch.upload([p.Q0 for p in probs])
    batch.integrate(Q, dts, 3)
    got = batch.download(Q)
    for p, g in zip(probs, got):
        sol = W.Solver(p.mesh)
        q = sol.upload(p.Q0)
        sol.integrate(q, p.S, p.dt, 3)
        assert np.array_equal(sol.download(q, p.S), g), p.mesh.K


def test_batch_matches_oracle(W, small):
    _print_case(test="batch-vs-oracle")
    probs, batch = small
    Q = batch.upload([p.Q0 for p in probs])
    batch.integrate(Q, [p.dt for p in probs], 2)
    got = batch.download(Q)
    for i in (0, 1, 5):   # 4, 16 and 49 elements
        p = probs[i]
        o = WADGOracle(p.mesh)
        for s in (0, p.S - 1):
            want = o.integrate(p.Q0[s], p.dt, 2)
            rel = np.linalg.norm(got[i][s] - want) / np.linalg.norm(want)
            mx = np.max(np.abs(got[i][s] - want)) / np.max(np.abs(want))
            assert rel <= 1e-12 and mx <= 1e-12, (i, s, rel, mx)


def test_schedules_and_tuner_bitwise_invariant(W, small):
    """Item schedules (split and persistent kernels, both orders), runs of
    the pipelined kernel (one slice each, three, and the default sixteen:
    runs of one slice have no prefetch, sixteen cover whole problems) and the
    tuner's choice all give the same bits."""
    _print_case(test="batch-schedules")
    probs, batch = small
    dts = [p.dt for p in probs]
    outs = []
    for wg, order, runs in ((2, 0, 0), (0, 0, 0), (1, 1, 0), (8, 1, 0), (4, 0, 0), (0, 0, 1),
                            (0, 0, 3), (0, 0, 16)):
        batch.set_schedule(wg, order)
        batch.set_runs(runs)
        Q = batch.upload([p.Q0 for p in probs])
        batch.integrate(Q, dts, 3)
        outs.append(batch.download(Q))
    Q0 = batch.upload([p.Q0 for p in probs])
    wg, order, runs, us = batch.tune(Q0, dts, reps=2)
    assert wg in (0, 1, 2, 4, 8) and order in (0, 1) and runs in (0, 4, 8, 16, 32, 128)
    assert us > 0
    assert np.array_equal(Q0.cpu().numpy(), batch.upload([p.Q0 for p in probs]).cpu().numpy())
    batch.integrate(Q0, dts, 3)
    outs.append(batch.download(Q0))
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)
    batch.set_runs(16)         # the default


def test_graph_replays_equal_eager(W, small):
    import torch
    _print_case(test="batch-graph")
    probs, batch = small
    dts = [p.dt for p in probs]
    Qe = batch.upload([p.Q0 for p in probs])
    Qg = batch.upload([p.Q0 for p in probs])
    we, wg = batch.workspace(), batch.workspace()
    batch.capture(Qg, wg, dts, 1)
    try:
        for r in range(3):
            batch.integrate(Qe, dts, 1, work=we)          # eager work between replays
            torch.cuda.synchronize()
            batch.replay()
            torch.cuda.synchronize()
            # padding lanes are unspecified on output; compare the problems' values
            for a, b in zip(batch.download(Qe), batch.download(Qg)):
                assert np.array_equal(a, b), r
    finally:
        batch.release_graph()


def test_graph_keeps_its_dt_when_eager_calls_change_it(W, small):
    """A captured graph records the sweep for the dt given at capture: an
    eager integrate with other dt between capture and replay (on another,
    non-blocking stream) changes neither the graph's result nor its own."""
    import torch
    _print_case(test="batch-graph-dt")
    probs, batch = small
    dt_a = [p.dt for p in probs]
    dt_b = [0.5 * p.dt for p in probs]
    want_b = batch.upload([p.Q0 for p in probs])
    batch.integrate(want_b, dt_b, 2)
    want_a = batch.upload([p.Q0 for p in probs])
    batch.integrate(want_a, dt_a, 2)                  # the eager tables now hold dt_a
    torch.cuda.synchronize()
    Qg, wg = batch.upload([p.Q0 for p in probs]), batch.workspace()
    Qe, we = batch.upload([p.Q0 for p in probs]), batch.workspace()
    side = torch.cuda.Stream()
    batch.capture(Qg, wg, dt_a, 2)
    try:
        batch.integrate(Qe, dt_b, 2, work=we, stream=side)   # rewrites the eager dt
        batch.replay(stream=side)
        torch.cuda.synchronize()
        for a, b in zip(batch.download(Qg), batch.download(want_a)):
            assert np.array_equal(a, b)
        for a, b in zip(batch.download(Qe), batch.download(want_b)):
            assert np.array_equal(a, b)
    finally:
        batch.release_graph()


def test_recapture_and_release_with_replays_queued(W, small):
    """A new capture replaces a graph whose replays are still queued on
    another stream, and a release frees one with a replay queued: both wait
    for the device to drain, so every queued replay runs whole."""
    import torch
    _print_case(test="batch-graph-recapture")
    probs, batch = small
    dts = [p.dt for p in probs]
    want2 = batch.upload([p.Q0 for p in probs])
    batch.integrate(want2, dts, 2)
    want4 = batch.upload([p.Q0 for p in probs])
    batch.integrate(want4, dts, 4)
    torch.cuda.synchronize()
    Qg, wg = batch.upload([p.Q0 for p in probs]), batch.workspace()
    Qh, wh = batch.upload([p.Q0 for p in probs]), batch.workspace()
    side = torch.cuda.Stream()
    try:
        batch.capture(Qg, wg, dts, 1)
        batch.replay(stream=side)
        batch.replay(stream=side)                  # queued, not waited for
        batch.capture(Qh, wh, dts, 2)              # replaces the graph
        batch.replay(stream=side)
        batch.replay(stream=side)
        batch.release_graph()                      # with a replay queued
        torch.cuda.synchronize()
        for a, b in zip(batch.download(Qg), batch.download(want2)):
            assert np.array_equal(a, b)
        for a, b in zip(batch.download(Qh), batch.download(want4)):
            assert np.array_equal(a, b)
    finally:
        batch.release_graph()


def test_full_batch_sampled_problems(W):
    import torch
    _print_case(test="batch-full", problems=1000)
    probs = make_batch()
    batch = W.Batch([p.mesh for p in probs], [p.S for p in probs])
    dts = [p.dt for p in probs]
    Q = batch.upload([p.Q0 for p in probs])
    batch.integrate(Q, dts, 1)
    torch.cuda.synchronize()
    Ks = np.array([p.mesh.K for p in probs])
    picks = [int(np.argmin(Ks)), int(np.argmax(Ks)), int(np.argsort(Ks)[500]), 999]
    got = batch.download(Q, picks)
    for i, g in zip(picks, got):
        p = probs[i]
        sol = W.Solver(p.mesh)
        q = sol.upload(p.Q0)
        sol.integrate(q, p.S, p.dt, 1)
        assert np.array_equal(sol.download(q, p.S), g), i


@pytest.mark.parametrize("N,nq1", [(1, 2), (2, 4), (4, 6)])
def test_other_degrees_all_batch_kernels(W, N, nq1):
    """Batches of other degrees and quadratures, mixing packed (4 and 9
    elements) and multi-group (100 elements) meshes with c^2 varying: every
    problem equals the single-problem path bitwise, with the split-work
    kernel (one workgroup per item), with persistent workgroups and, where
    it fits, with the pipelined kernel (refused with UNSUPPORTED at N = 4)."""
    from workloads import periodic_quad_mesh, c2_layered
    _print_case(test="batch-degrees", N=N, nq1=nq1)
    meshes = [periodic_quad_mesh(k, N, eps=0.05, warp="skew", rotate_seed=k) for k in (2, 3, 10)]
    S = [5, 3, 2]
    rng = np.random.default_rng(N)
    Q0 = [rng.standard_normal((s, 3, m.Np, m.K)) for m, s in zip(meshes, S)]
    dts = [0.1 / (m.K1D * (N + 1) ** 2) for m in meshes]
    batch = W.Batch(meshes, S, nq1=nq1, c2=c2_layered)
    assert max(batch.pack) > 1 and min(batch.pack) == 1
    outs = []
    for wg in (0, 2):
        batch.set_schedule(wg, 0)
        Q = batch.upload(Q0)
        batch.integrate(Q, dts, 2)
        outs.append(batch.download(Q))
    if N <= 2:      # the pipelined kernel's LDS plan fits
        batch.set_runs(2)
        Q = batch.upload(Q0)
        batch.integrate(Q, dts, 2)
        outs.append(batch.download(Q))
    else:
        with pytest.raises(W.WadgError) as e:
            batch.set_runs(2)
        assert e.value.status == W.binding.WADG_E_UNSUPPORTED
    for i, (m, s) in enumerate(zip(meshes, S)):
        sol = W.Solver(m, nq1=nq1, c2=c2_layered)
        q = sol.upload(Q0[i])
        sol.integrate(q, s, dts[i], 2)
        want = sol.download(q, s)
        assert np.all(np.isfinite(want))
        assert np.array_equal(outs[0][i], want), (i, "split")
        assert np.array_equal(outs[1][i], want), (i, "persistent")
        if N <= 2:
            assert np.array_equal(outs[2][i], want), (i, "pipelined")
