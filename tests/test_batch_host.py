"""Batch (many independent problems) pieces that need no GPU: the packed
layout helpers, the workload generator's subset consistency, and the
batch C ABI's argument validation, which runs before any HIP call."""

import numpy as np
import pytest

from workloads import batch_shapes, make_batch, periodic_quad_mesh

W = pytest.importorskip("paper_1608_03836_amd.binding",
                        reason="libwadg.so not built (run __graft_entry__.build())")


@pytest.mark.parametrize("S,K,P", [(1, 4, 16), (7, 9, 7), (34, 4, 16), (5, 36, 1), (3, 81, 1),
                                   (16, 16, 4), (109, 36, 7), (114, 225, 3), (40, 81, 13)])
def test_pack_round_trip(S, K, P):
    rng = np.random.default_rng(S * 100 + K)
    Q = rng.standard_normal((S, 3, 16, K))
    v = W.pack_batch_problem(Q, P)
    Sv = -(-S // P)
    G = -(-(P * K) // 64)
    assert v.size == Sv * G * 3 * 16 * 64
    assert np.array_equal(W.unpack_batch_problem(v, S, K, 16, P), Q)
    # slice s, element k sits in virtual slice s // P at virtual element (s % P) K + k
    s, k = S - 1, K - 1
    t = v.reshape(Sv, G, 3, 16, 64)
    e = (s % P) * K + k
    assert t[s // P, e // 64, 2, 5, e % 64] == Q[s, 2, 5, k]


def test_batch_workload_shapes_and_subsets():
    k1d, S, _ = batch_shapes()
    assert len(k1d) == 1000 and k1d.min() == 2 and k1d.max() == 16
    assert S.min() >= 8 and S.max() <= 128
    a = make_batch(count=6)
    b = make_batch(members=[5])
    assert a[5].S == b[0].S and a[5].mesh.K == b[0].mesh.K and a[5].dt == b[0].dt
    assert np.array_equal(a[5].Q0, b[0].Q0)
    # slice s starts from the exact solution at t = 4 s dt
    m = a[0]
    p, u, v = m.exact(m.mesh.x, m.mesh.y, 4 * 3 * m.dt)
    assert np.allclose(m.Q0[3, 0], p.T) and np.allclose(m.Q0[3, 1], u.T)


def _desc(m, N=None, nq1=None):
    return W.MeshDesc(m.N if N is None else N, (m.N + 2) if nq1 is None else nq1, m.x, m.y,
                      m.etoe, m.etof)


def test_batch_create_validates_before_device_work():
    import ctypes
    m2 = periodic_quad_mesh(2, 3)
    m3 = periodic_quad_mesh(3, 3)
    with pytest.raises(W.WadgError) as e:
        W.wadg_batch_create([_desc(m2), _desc(m3, nq1=4)], [4, 4])
    assert e.value.status == W.WADG_E_INVALID
    with pytest.raises(W.WadgError) as e:
        W.wadg_batch_create([_desc(m2), _desc(m3)], [4, 0])
    assert e.value.status == W.WADG_E_INVALID
    x = m3.x.copy()
    x[4] = x[4].reshape(4, 4)[:, ::-1].reshape(-1)          # mirrored element: J < 0
    bad = W.MeshDesc(3, 5, x, m3.y, m3.etoe, m3.etof)
    with pytest.raises(W.WadgError) as e:
        W.wadg_batch_create([_desc(m2), bad], [4, 4])
    assert e.value.status == W.WADG_E_GEOMETRY and "problem 1" in W.wadg_last_error()
    assert W.LIB.wadg_batch_create(None, 1, None, 0, ctypes.byref(ctypes.c_void_p())) \
        == W.WADG_E_INVALID
    assert W.LIB.wadg_batch_integrate(None, None, None, None, 1, None) == W.WADG_E_INVALID
    assert W.LIB.wadg_batch_replay(None, None) == W.WADG_E_INVALID
    assert W.LIB.wadg_batch_set_runs(None, 4) == W.WADG_E_INVALID
    W.LIB.wadg_batch_destroy(None)
