"""Maximum-size GPU parity: a mesh at the size limit of one slice, every
element of every slice checked.

The mesh is the 147 x 147 periodic cover of a 16 x 16 curvilinear mesh (N = 3,
nq1 = 5, skew warp, rotated local frames, heterogeneous c^2): K = 2352^2 =
5,531,904 elements in 86,436 groups of 64, so one FP64 slice of the tiled
state is 2.124e9 bytes, 98.9 % of the 2 GiB a slice may take.  Ten slices
make state arrays of 2.66e9 doubles (21 GB), past 2^31 values and 2^34
bytes.

Every copy in the cover keeps its base element's coordinates, frame and c^2,
so a state that repeats the base state on each copy evolves copy by copy as
the base state does (pinned on the oracle by
test_oracle_wadg.test_periodic_cover_evolves_copy_by_copy).  Each element's
arithmetic in the kernels depends only on its own lane, geometry and the
neighbour values it gathers, never on where it sits, so the cover's results
must equal the base mesh's GPU results copied, bitwise; and the base mesh's
GPU results are checked against the oracle at the FP64 bar (1e-12) and the
FP32-bulk bar (1e-6).  The copies and comparisons run on the device (torch
gathers); all arithmetic of the method runs in the library.
"""

import numpy as np
import pytest

from workloads import periodic_quad_mesh, periodic_cover, c2_layered
from oracle import WADGOracle

pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL_FP32 = 1e-6
N, NQ1, BASE_K1D, COPIES = 3, 5, 16, 147
S, NSTEPS, DT = 10, 3, 1.0 / 512     # dt K1D = 1/32 on the base mesh, as the workloads use


def _say(msg):
    print("CASE max-size", msg, flush=True)


class _Max:
    pass


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1608_03836_amd as W
    B = W.binding
    m = _Max()
    m.torch, m.W = torch, W
    dev = torch.device("cuda", 0)
    base = periodic_quad_mesh(BASE_K1D, N, eps=0.05, warp="skew", rotate_seed=11)
    xq, yq = B.wadg_quadrature_points(B.MeshDesc(N, NQ1, base.x, base.y, base.etoe, base.etof))
    c2b = c2_layered(xq, yq)
    m.small = W.Solver(base, nq1=NQ1, c2q=c2b)
    cover, idx = periodic_cover(base, COPIES)
    m.K = cover.K
    m.G = (m.K + 63) // 64
    slice_bytes = m.G * 3 * (N + 1) ** 2 * 64 * 8
    assert 0.98 * 2 ** 31 < slice_bytes < 2 ** 31
    assert S * slice_bytes // 8 > 2 ** 31
    _say(f"K={m.K} groups={m.G} S={S} slice_bytes={slice_bytes}: wadg_create")
    m.big = W.Solver(cover, nq1=NQ1, c2q=c2b[idx])
    del cover
    pad = np.full(m.G * 64, base.K, dtype=np.int64)    # padding lanes -> a zero column
    pad[:m.K] = idx
    m.idx = torch.from_numpy(pad).to(dev)
    _say("oracle on the base mesh")
    m.Q0 = np.random.default_rng(2024).standard_normal((S, 3, (N + 1) ** 2, base.K))
    o = WADGOracle(base, nq1=NQ1, c2=c2_layered)
    m.or_rhs = o.rhs(m.Q0)
    m.or_int = o.integrate(m.Q0, DT, NSTEPS)
    m.oracle = o
    m.dev = dev
    yield m
    m.big.close()
    m.small.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _expand(m, Qn):
    """Base natural state [S][3][Np][Kb] (host or device) -> the cover's tiled
    state on the device, every copy holding the base state."""
    t = m.torch
    src = t.as_tensor(np.asarray(Qn) if not t.is_tensor(Qn) else Qn, device=m.dev)
    src = t.cat([src, src.new_zeros(src.shape[:3] + (1,))], dim=3)
    Np = src.shape[2]
    out = t.empty((src.shape[0], m.G, 3, Np, 64), dtype=src.dtype, device=m.dev)
    for s in range(src.shape[0]):
        out[s].copy_(src[s][:, :, m.idx].view(3, Np, m.G, 64).permute(2, 0, 1, 3))
    return out.reshape(-1)


def _small_natural(m, Qt):
    """Base tiled device state -> natural [S][3][Np][Kb] device tensor."""
    Np = (N + 1) ** 2
    Kb = m.small.K
    Gb = (Kb + 63) // 64
    v = Qt.view(-1, Gb, 3, Np, 64).permute(0, 2, 3, 1, 4).reshape(-1, 3, Np, Gb * 64)
    return v[..., :Kb]


def _compare(m, Qbig, small_gpu_t, oracle, tol):
    """Each slice of the cover's tiled state against the copied base GPU state
    (bitwise) and the copied oracle state (relative l2 and max error)."""
    t = m.torch
    Np = (N + 1) ** 2
    sg = _small_natural(m, small_gpu_t)
    orc = t.as_tensor(oracle, device=m.dev)
    v = Qbig.view(S, m.G, 3, Np, 64)
    worst = 0.0
    for s in range(S):
        got = v[s].permute(1, 2, 0, 3).reshape(3, Np, m.G * 64)[..., :m.K]
        z = sg[s][:, :, m.idx[:m.K]]
        assert t.equal(got, z), f"slice {s}: not the copied base result"
        w = orc[s][:, :, m.idx[:m.K]]
        d = got - w
        rel = (t.linalg.vector_norm(d) / t.linalg.vector_norm(w)).item()
        mx = (d.abs().max() / w.abs().max()).item()
        assert rel <= tol and mx <= tol, f"slice {s}: rel {rel:.3e}, max {mx:.3e}"
        worst = max(worst, rel, mx)
        del got, z, w, d
    return worst


def test_max_size_rhs(M):
    """dQ/dt (Section 4's load vector and WADG mass inverse) on the cover."""
    _say(f"rhs kernel={M.big.kernel_in_use(rhs=True)}")
    Qb = _expand(M, M.Q0)
    out = M.big.rhs(Qb, S)
    qs = M.small.upload(M.Q0)
    outs = M.small.rhs(qs, S)
    M.torch.cuda.synchronize()
    worst = _compare(M, out, outs, M.or_rhs, TOL)
    print(f"max-size rhs: worst relative error vs oracle {worst:.3e}")
    del Qb, out


def test_max_size_sweep_and_norms(M):
    """NSTEPS LSRK(5,4) steps of all S slices in the launch configuration of
    the default sweep, then the per-slice norms against the oracle state."""
    _say(f"sweep kernel={M.big.kernel_in_use()}")
    Qb = _expand(M, M.Q0)
    M.big.integrate(Qb, S, DT, NSTEPS)
    qs = M.small.upload(M.Q0)
    M.small.integrate(qs, S, DT, NSTEPS)
    M.torch.cuda.synchronize()
    worst = _compare(M, Qb, qs, M.or_int, TOL)
    print(f"max-size sweep: worst relative error vs oracle {worst:.3e}")
    _say("norms")
    nb = M.big.norms(Qb, None, S)
    ns = M.small.norms(qs, None, S)
    assert np.all(nb[:, 3] == 1.0)
    assert np.all(nb[:, 2] == ns[:, 2])                 # max |Q_s|: same values
    np.testing.assert_allclose(nb[:, 0], COPIES * ns[:, 0], rtol=TOL, atol=0)
    want = _expand(M, M.or_int)
    nd = M.big.norms(Qb, want, S)
    assert np.all(nd[:, 0] <= TOL * nd[:, 1]), nd[:, 0] / nd[:, 1]
    np.testing.assert_allclose(nd[:, 1], COPIES * np.linalg.norm(M.or_int.reshape(S, -1), axis=1),
                               rtol=TOL, atol=0)
    _say("L2 norms")
    nl = M.big.l2_norms(Qb, want, S)
    o_l2 = np.array([M.oracle.l2_norm(M.or_int[s]) for s in range(S)])
    np.testing.assert_allclose(nl[:, 1], COPIES * o_l2, rtol=TOL, atol=0)
    assert np.all(nl[:, 0] <= TOL * nl[:, 1]), nl[:, 0] / nl[:, 1]
    np.testing.assert_allclose(M.big.l2_norms(Qb, None, S)[:, 0],
                               COPIES * M.small.l2_norms(qs, None, S)[:, 0], rtol=TOL, atol=0)
    del Qb, want


def test_max_size_fp32_bulk(M):
    """The FP32-bulk sweep (FP64 state in and out) on the cover."""
    _say(f"fp32 kernel={M.big.kernel_in_use(fp32=True)}")
    Qb = _expand(M, M.Q0)
    M.big.integrate_fp32(Qb, S, DT, NSTEPS)
    qs = M.small.upload(M.Q0)
    M.small.integrate_fp32(qs, S, DT, NSTEPS)
    M.torch.cuda.synchronize()
    worst = _compare(M, Qb, qs, M.or_int, TOL_FP32)
    print(f"max-size FP32 bulk: worst relative error vs oracle {worst:.3e}")
    del Qb
