"""GPU: wadg_norms_noalloc, the reduction for callers that cannot allocate,
through the C ABI.  It runs wadg_norms' kernels in the library's static
per-device scratch, so its output equals wadg_norms' (with caller scratch)
bit for bit: on two calls in a row, the second with fewer slices and other
data (the array keeps the first call's contents), with and without B, with
a non-finite entry, and it refuses more slices than its scratch holds
before any HIP call."""

import numpy as np
import pytest

from workloads import periodic_quad_mesh

pytestmark = pytest.mark.gpu


def test_noalloc_norms_equal_caller_scratch_norms():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_1608_03836_amd as W
    from paper_1608_03836_amd import binding as B
    print("CASE test=norms-noalloc", flush=True)
    mesh = periodic_quad_mesh(9, 3, eps=0.05)       # 81 elements: a full and a ragged group
    sol = W.Solver(mesh)
    rng = np.random.default_rng(11)
    scratch = torch.empty(B.wadg_norms_workspace_bytes(sol.ctx, 9) // 8, dtype=torch.float64,
                          device="cuda")
    for S in (9, 4):                                # second call: fewer slices, other data
        A = sol.upload(rng.standard_normal((S, 3, mesh.Np, mesh.K)))
        Bv = sol.upload(rng.standard_normal((S, 3, mesh.Np, mesh.K)))
        for other in (Bv, None):
            want = B.wadg_norms(sol.ctx, A, other, S, scratch)
            got = B.wadg_norms_noalloc(sol.ctx, A, other, S)
            assert np.array_equal(got, want), (S, other is None)
        # and both are the norms of the downloaded arrays (B = None last)
        a, b = sol.download(A, S), sol.download(Bv, S)
        assert np.allclose(got[:, 0], np.linalg.norm(a.reshape(S, -1), axis=1), rtol=1e-13,
                           atol=0)
        got_d = B.wadg_norms_noalloc(sol.ctx, A, Bv, S)
        assert np.allclose(got_d[:, 0], np.linalg.norm((a - b).reshape(S, -1), axis=1),
                           rtol=1e-13, atol=0)
    # a non-finite entry: flagged as by wadg_norms
    A = sol.upload(rng.standard_normal((2, 3, mesh.Np, mesh.K)))
    A.view(-1)[5] = float("nan")
    got = B.wadg_norms_noalloc(sol.ctx, A, None, 2, check_finite=False)
    want = B.wadg_norms(sol.ctx, A, None, 2, scratch, check_finite=False)
    assert np.array_equal(np.isnan(got), np.isnan(want))
    assert np.array_equal(got[:, 3], want[:, 3]) and got[0, 3] == 0.0 and got[1, 3] == 1.0
    with pytest.raises(W.WadgError) as e:
        B.wadg_norms_noalloc(sol.ctx, A, None, 2)
    assert e.value.status == B.WADG_E_NONFINITE
    # more slices than the static scratch holds: refused before any launch
    with pytest.raises(W.WadgError, match="static scratch") as e:
        B.wadg_norms_noalloc(sol.ctx, A.data_ptr(), None, B.WADG_NORMS_NOALLOC_MAX_S + 1)
    assert e.value.status == B.WADG_E_INVALID
    torch.cuda.synchronize()
