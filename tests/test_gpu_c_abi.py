"""GPU: the library through its C ABI alone.  A plain C program
(paper_1608_03836_amd/csrc/abi_demo.c, linked against libwadg.so by the
build) reads a mesh and tiled start states, creates a context, integrates
every slice and takes the norms -- no Python and no torch in that process.
Its result equals the Python binding's bit for bit (same kernels, same
launches) and the oracle's to the FP64 bar, for the automatic kernel choice
and for the streamed kernel."""

import os
import subprocess

import numpy as np
import pytest

from workloads import periodic_quad_mesh
from oracle import WADGOracle

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEMO = os.path.join(ROOT, "paper_1608_03836_amd", "abi_demo")


@pytest.mark.parametrize("kernel", [0, 1])
def test_c_consumer_matches_python_binding_and_oracle(tmp_path, kernel):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1608_03836_amd as W
    from paper_1608_03836_amd import binding as B
    assert os.path.exists(DEMO), "abi_demo is built with the library (build.py)"
    print(f"CASE test=c-abi kernel={kernel}", flush=True)
    N, K1D, S, nsteps = 3, 9, 3, 2
    mesh = periodic_quad_mesh(K1D, N, eps=0.05, warp="skew", rotate_seed=4)
    dt = 0.1 / (K1D * (N + 1) ** 2)
    Q0 = np.random.default_rng(31).standard_normal((S, 3, mesh.Np, mesh.K))
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(np.array([N, N + 2, mesh.K, S, nsteps, kernel], dtype="<i4").tobytes())
        f.write(np.array([dt, 1.0, 1.0], dtype="<f8").tobytes())
        for a, t in ((mesh.x, "<f8"), (mesh.y, "<f8"), (mesh.etoe, "<i4"), (mesh.etof, "<i4")):
            f.write(np.ascontiguousarray(a, dtype=t).tobytes())
        f.write(B.tile_state(Q0).astype("<f8").tobytes())
    p = subprocess.run([DEMO, str(inp), str(out)], capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, p.stderr
    raw = np.fromfile(out, dtype="<f8")
    sol = W.Solver(mesh)
    sol.set_kernel(kernel)
    n = S * sol.slice_doubles
    got = sol.download(torch.from_numpy(raw[:n]), S)
    norms = raw[n:].reshape(S, 4)
    Q = sol.upload(Q0)
    sol.integrate(Q, S, dt, nsteps)
    want_py = sol.download(Q, S)
    assert np.array_equal(got, want_py)
    assert np.array_equal(norms, sol.norms(Q, None, S))
    want = WADGOracle(mesh).integrate(Q0, dt, nsteps)
    for s in range(S):
        rel = np.linalg.norm(got[s] - want[s]) / np.linalg.norm(want[s])
        assert rel <= 1e-12, (s, rel)


def test_binding_refuses_unusable_tensors():
    """The Python binding checks every device tensor against the call it is
    passed to before the library sees its pointer: too small, on the host,
    or not float64 where a state is expected is a ValueError, and so is a
    host array of per-problem values of the wrong length.  Nothing is
    launched in these cases."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1608_03836_amd as W
    print("CASE test=binding-refusals", flush=True)
    mesh = periodic_quad_mesh(4, 2, eps=0.05)
    sol = W.Solver(mesh)
    S, dt = 3, 1e-3
    Q, work = sol.empty_state(S), sol.workspace(S)
    with pytest.raises(ValueError, match="Q holds"):
        sol.integrate(Q[:-1], S, dt, 1, work=work)
    with pytest.raises(ValueError, match="work holds"):
        sol.integrate(Q, S, dt, 1, work=work[:-1])
    with pytest.raises(ValueError, match="device tensor"):
        sol.integrate(Q.cpu(), S, dt, 1, work=work)
    with pytest.raises(ValueError, match="float64"):
        sol.rhs(Q.float(), S)
    with pytest.raises(ValueError, match="dQdt holds"):
        sol.rhs(Q, S, out=sol.empty_state(S - 1))
    with pytest.raises(ValueError, match="B holds"):
        sol.norms(Q, Q[:7], S)
    with pytest.raises(ValueError, match="A holds"):
        sol.l2_norms(Q[:7], None, S)
    with pytest.raises(ValueError, match="work holds"):
        sol.integrate_fp32(Q, S, dt, 1, work=sol.workspace_fp32(S)[:-1])
    with pytest.raises(ValueError, match="chk holds"):
        sol.adjoint(sol.empty_state(S), sol.empty_state(1), S, dt, 1)
    meshes = [periodic_quad_mesh(k, 2, eps=0.05) for k in (2, 3)]
    with pytest.raises(ValueError, match="one slice count per mesh"):
        W.Batch(meshes, [2])
    batch = W.Batch(meshes, [2, 3])
    Qb, wb = batch.upload([np.zeros((s, 3, m.Np, m.K)) for m, s in zip(meshes, (2, 3))]), \
        batch.workspace()
    with pytest.raises(ValueError, match="dt holds"):
        batch.integrate(Qb, [dt], 1, work=wb)
    with pytest.raises(ValueError, match="Q holds"):
        batch.integrate(Qb[:-1], [dt, dt], 1, work=wb)
    batch.integrate(Qb, [dt, dt], 1, work=wb)        # the well-formed call runs
    torch.cuda.synchronize()


def test_reductions_take_caller_scratch():
    """wadg_norms and wadg_l2_norms run in caller-owned device scratch: the
    size queries give S (64 x 4 + 4) and 2 S (ceil(K/64) + 1) doubles, a
    buffer one byte short, a missing one or one that overlaps an operand is
    refused before any launch, and a buffer of exactly the queried size
    gives the same sums as a larger one."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1608_03836_amd as W
    from paper_1608_03836_amd import binding as B
    print("CASE test=reduction-scratch", flush=True)
    mesh = periodic_quad_mesh(9, 3, eps=0.05)       # 81 elements: 2 groups
    sol = W.Solver(mesh)
    S = 5
    nb = B.wadg_norms_workspace_bytes(sol.ctx, S)
    lb = B.wadg_l2_norms_workspace_bytes(sol.ctx, S)
    assert nb == 8 * S * (64 * 4 + 4)
    assert lb == 8 * 2 * S * (2 + 1)
    Q = sol.upload(np.random.default_rng(3).standard_normal((S, 3, mesh.Np, mesh.K)))
    exact = torch.empty(nb // 8, dtype=torch.float64, device="cuda")
    big = torch.empty(nb // 8 + 1000, dtype=torch.float64, device="cuda")
    a = B.wadg_norms(sol.ctx, Q, None, S, exact)
    assert np.array_equal(a, B.wadg_norms(sol.ctx, Q, None, S, big))
    for fn, need in ((B.wadg_norms, nb), (B.wadg_l2_norms, lb)):
        with pytest.raises(W.WadgError, match="needed") as e:
            fn(sol.ctx, Q, None, S, big.data_ptr(), scratch_bytes=need - 1)
        assert e.value.status == B.WADG_E_INVALID
        with pytest.raises(W.WadgError, match="scratch must not be NULL"):
            fn(sol.ctx, Q, None, S, None)
        with pytest.raises(W.WadgError, match="overlap"):
            fn(sol.ctx, Q, None, S, Q.data_ptr(), scratch_bytes=need)
    la = B.wadg_l2_norms(sol.ctx, Q, None, S, big[: lb // 8])
    assert np.array_equal(la, sol.l2_norms(Q, None, S))
    torch.cuda.synchronize()
