"""C-ABI tests that need no GPU: the library loads and exports every symbol
the header declares, the host-side geometry agrees with the oracle's
independent (modal) construction, and invalid input is rejected with the
documented status codes before any HIP call."""

import os
import re

import numpy as np
import pytest

from workloads import periodic_quad_mesh, c2_layered
from oracle import WADGOracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wadg.h")

W = pytest.importorskip("paper_1608_03836_amd.binding",
                        reason="libwadg.so not built (run __graft_entry__.build())")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wadg_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    declared = _declared_functions()
    assert len(declared) >= 12
    for name in declared:
        assert hasattr(W.LIB, name), name
    assert set(declared) == set(W.EXPORTED)


def _mesh(K1D=4, N=3, warp="skew", rot=3, nq1=None):
    m = periodic_quad_mesh(K1D, N, eps=0.05, warp=warp, rotate_seed=rot)
    return m, W.MeshDesc(N, N + 2 if nq1 is None else nq1, m.x, m.y, m.etoe, m.etof)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_quadrature_points_match_oracle(N):
    m, d = _mesh(N=N)
    xq, yq = W.wadg_quadrature_points(d)
    o = WADGOracle(m, nq1=N + 2)
    assert np.max(np.abs(xq - o.xq)) < 1e-14
    assert np.max(np.abs(yq - o.yq)) < 1e-14


@pytest.mark.parametrize("N,dnq", [(1, 1), (2, 2), (3, 2), (3, 3), (4, 1)])
def test_geometry_matches_oracle(N, dnq):
    m, d0 = _mesh(N=N, nq1=N + dnq)
    xq, yq = W.wadg_quadrature_points(d0)
    d = W.MeshDesc(N, N + dnq, m.x, m.y, m.etoe, m.etof, c2_layered(xq, yq))
    vol, face = W.wadg_geometry(d)
    o = WADGOracle(m, nq1=N + dnq, c2=c2_layered)
    ref = o.ref
    xr, xs = o.cx @ ref.Vr.T, o.cx @ ref.Vs.T
    yr, ys = o.cy @ ref.Vr.T, o.cy @ ref.Vs.T
    Wq = ref.W[None]
    scale = np.max(np.abs(Wq * ys))
    for got, want in zip(vol[:4], (Wq * ys, -Wq * xs, -Wq * yr, Wq * xr)):
        assert np.max(np.abs(got.T - want)) < 1e-13 * scale
    assert np.max(np.abs(vol[4].T * o.J / o.c2q - 1)) < 1e-12
    assert np.max(np.abs(vol[5].T * o.J - 1)) < 1e-12
    for f in range(4):
        assert np.max(np.abs(face[0, f].T - o.nx[f])) < 1e-13
        assert np.max(np.abs(face[1, f].T - o.ny[f])) < 1e-13
        wsJ = ref.wf[None] * o.sJ[f]
        assert np.max(np.abs(face[2, f].T - wsJ)) < 1e-13 * np.max(wsJ)


def _status(fn, *args):
    with pytest.raises(W.WadgError) as e:
        fn(*args)
    return e.value.status


def test_rejects_bad_degree_and_quadrature():
    m, _ = _mesh(N=3)
    assert _status(W.wadg_geometry, W.MeshDesc(7, 8, m.x, m.y, m.etoe, m.etof)) == W.WADG_E_UNSUPPORTED
    assert _status(W.wadg_geometry, W.MeshDesc(3, 3, m.x, m.y, m.etoe, m.etof)) == W.WADG_E_UNSUPPORTED
    assert _status(W.wadg_geometry, W.MeshDesc(3, 7, m.x, m.y, m.etoe, m.etof)) == W.WADG_E_UNSUPPORTED


def test_rejects_inverted_element():
    m, _ = _mesh(N=2, rot=None)
    x = m.x.copy()
    n = 3
    x[5] = x[5].reshape(n, n)[:, ::-1].reshape(-1)       # mirror element 5: J < 0
    st = _status(W.wadg_geometry, W.MeshDesc(2, 4, x, m.y, m.etoe, m.etof))
    assert st == W.WADG_E_GEOMETRY
    assert "Jacobian" in W.wadg_last_error()


def test_rejects_nonconforming_and_asymmetric_connectivity():
    m, _ = _mesh(N=2)
    etoe = m.etoe.copy()
    etoe[0, 1] = (etoe[0, 1] + 1) % m.K
    assert _status(W.wadg_geometry, W.MeshDesc(2, 4, m.x, m.y, etoe, m.etof)) == W.WADG_E_GEOMETRY
    etof = m.etof.copy()
    etof[3, 2] ^= 4                                       # flip bit on one side only
    assert _status(W.wadg_geometry, W.MeshDesc(2, 4, m.x, m.y, m.etoe, etof)) == W.WADG_E_GEOMETRY
    etoe = m.etoe.copy()
    etoe[2, 0] = m.K + 5
    assert _status(W.wadg_geometry, W.MeshDesc(2, 4, m.x, m.y, etoe, m.etof)) == W.WADG_E_INVALID


def test_rejects_bad_wavespeed_and_penalty():
    m, d = _mesh(N=2)
    c2q = np.ones((m.K, 16))
    c2q[1, 3] = -1.0
    assert _status(W.wadg_geometry, W.MeshDesc(2, 4, m.x, m.y, m.etoe, m.etof, c2q)) == W.WADG_E_INVALID
    c2q[1, 3] = np.nan
    assert _status(W.wadg_geometry, W.MeshDesc(2, 4, m.x, m.y, m.etoe, m.etof, c2q)) == W.WADG_E_INVALID
    bad = W.MeshDesc(2, 4, m.x, m.y, m.etoe, m.etof, tau_p=-1.0)
    assert _status(W.wadg_geometry, bad) == W.WADG_E_INVALID


def test_rejects_non_finite_coordinates():
    m, _ = _mesh(N=2)
    x = m.x.copy()
    x[4, 2] = np.inf
    assert _status(W.wadg_geometry, W.MeshDesc(2, 4, x, m.y, m.etoe, m.etof)) == W.WADG_E_GEOMETRY


def test_null_arguments():
    import ctypes
    assert W.LIB.wadg_geometry(None, None, None) == W.WADG_E_INVALID
    assert W.LIB.wadg_create(None, 0, ctypes.byref(ctypes.c_void_p())) == W.WADG_E_INVALID
    assert W.LIB.wadg_rhs(None, None, None, 1, None) == W.WADG_E_INVALID
    assert W.LIB.wadg_integrate(None, None, None, 1, 0.1, 1, None) == W.WADG_E_INVALID
    assert W.LIB.wadg_norms(None, None, None, 1, None, 0, None, None) == W.WADG_E_INVALID
    assert W.LIB.wadg_l2_norms(None, None, None, 1, None, 0, None, None) == W.WADG_E_INVALID
    assert W.LIB.wadg_norms_workspace_bytes(None, 1, None) == W.WADG_E_INVALID
    assert W.LIB.wadg_l2_norms_workspace_bytes(None, 1, None) == W.WADG_E_INVALID
    assert W.LIB.wadg_workspace_bytes(None, 1, None) == W.WADG_E_INVALID
    W.LIB.wadg_destroy(None)
    for st in (0, -1, -2, -3, -4, -5, -99):
        assert W.wadg_status_string(st)


def test_tiled_layout_round_trip():
    rng = np.random.default_rng(1)
    for K in (1, 63, 64, 65, 200):
        Q = rng.standard_normal((3, 3, 9, K))
        t = W.tile_state(Q)
        assert t.shape == (3, (K + 63) // 64, 3, 9, 64)
        assert np.array_equal(W.untile_state(t, K), Q)
        # element k = 64 g + l, field f, node n sits at t[s, g, f, n, l]
        k = K - 1
        assert t[2, k // 64, 1, 4, k % 64] == Q[2, 1, 4, k]


def test_single_hip_runtime_in_process():
    """The binding and torch share one libamdhip64 (two runtimes in one
    process break device selection)."""
    import torch  # noqa: F401
    maps = open("/proc/self/maps").read()
    libs = {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}
    assert len(libs) == 1, libs


def test_geometry_of_periodic_cover_repeats_base_geometry():
    """Host geometry depends only on an element's own coordinates and c^2, so
    on a periodic cover (copies of the base mesh with unchanged coordinates)
    every copy's geometry equals its base element's, bitwise; the cover's
    wrap-around faces match modulo the period."""
    from workloads import periodic_cover
    m, d = _mesh(K1D=5, N=2, rot=8, nq1=4)
    cov, idx = periodic_cover(m, 3)
    dc = W.MeshDesc(2, 4, cov.x, cov.y, cov.etoe, cov.etof)
    xq, yq = W.wadg_quadrature_points(d)
    c2 = c2_layered(xq, yq)
    vb, fb = W.wadg_geometry(W.MeshDesc(2, 4, m.x, m.y, m.etoe, m.etof, c2))
    vc, fc = W.wadg_geometry(W.MeshDesc(2, 4, cov.x, cov.y, cov.etoe, cov.etof, c2[idx]))
    assert np.array_equal(vc, vb[..., idx]) and np.array_equal(fc, fb[..., idx])
    assert np.array_equal(W.wadg_quadrature_points(dc)[0], xq[idx])


def test_mesh_arrays_of_the_wrong_shape_are_refused():
    """The binding checks array shapes before the library reads them."""
    m, d = _mesh(N=2, nq1=4)
    with pytest.raises(ValueError, match="c2q"):
        W.MeshDesc(2, 4, m.x, m.y, m.etoe, m.etof, np.ones((m.K, 9)))
    with pytest.raises(ValueError, match="etof"):
        W.MeshDesc(2, 4, m.x, m.y, m.etoe, m.etof[:, :3])
    with pytest.raises(ValueError, match="y"):
        W.MeshDesc(2, 4, m.x, m.y[:-1], m.etoe, m.etof)


def test_cfl_number_of_affine_and_curved_meshes():
    """wadg_cfl_number: on an affine K1D x K1D mesh of the unit torus with
    c^2 = 1 the element size is exactly 1/K1D, so nu = dt (N+1)^2 K1D; with
    c^2 = gamma c0^2 the speed is sqrt(gamma max c0^2) over the volume
    points (NumPy over wadg_quadrature_points); a curved mesh has smaller
    elements somewhere, so a larger nu; bad arguments are refused."""
    for N in (1, 3):
        m = periodic_quad_mesh(6, N, eps=0.0)
        d = W.MeshDesc(N, N + 2, m.x, m.y, m.etoe, m.etof)
        nu = W.wadg_cfl_number(d, 1e-3)
        assert abs(nu - 1e-3 * (N + 1) ** 2 * 6) <= 1e-13 * nu
        xq, yq = W.wadg_quadrature_points(d)
        c2 = c2_layered(xq, yq)
        dc = W.MeshDesc(N, N + 2, m.x, m.y, m.etoe, m.etof, c2)
        nu2 = W.wadg_cfl_number(dc, 1e-3, 1.7)
        assert abs(nu2 - nu * np.sqrt(1.7 * c2.max())) <= 1e-13 * nu2
        mc = periodic_quad_mesh(6, N, eps=0.05)
        assert W.wadg_cfl_number(W.MeshDesc(N, N + 2, mc.x, mc.y, mc.etoe, mc.etof), 1e-3) > nu
    for dt, sc in ((0.0, 1.0), (-1.0, 1.0), (np.inf, 1.0), (1e-3, 0.0), (1e-3, np.nan)):
        assert _status(W.wadg_cfl_number, d, dt, sc) == W.WADG_E_INVALID
    assert W.LIB.wadg_cfl_number(None, 1e-3, 1.0, None) == W.WADG_E_INVALID


@pytest.mark.parametrize("N,warp,tau,c2", [(1, "skew", 1.0, None), (2, "skew", 1.0, None),
                                           (3, "skew", 1.0, None), (3, "diag", 0.0, "layered"),
                                           (4, "skew", 1.0, None)])
def test_cfl_bound_is_inside_the_stability_region(N, warp, tau, c2):
    """The parareal coarse-step bound: at nu = WADG_CFL_MAX (the library's
    CFL number of the step) every eigenvalue lambda of the assembled WADG
    operator (the oracle's, curved periodic 4 x 4 meshes) satisfies
    |R(dt lambda)| <= 1 for the stability polynomial R of the LSRK(5,4)
    scheme, so the coarse sweep does not grow."""
    from oracle.lsrk import stability_polynomial_coeffs
    c2f = c2_layered if c2 == "layered" else None
    m = periodic_quad_mesh(4, N, eps=0.05, warp=warp)
    d = W.MeshDesc(N, N + 2, m.x, m.y, m.etoe, m.etof)
    if c2f is not None:
        xq, yq = W.wadg_quadrature_points(d)
        d = W.MeshDesc(N, N + 2, m.x, m.y, m.etoe, m.etof, c2f(xq, yq))
    dt = W.WADG_CFL_MAX / W.wadg_cfl_number(d, 1.0)
    lam = np.linalg.eigvals(WADGOracle(m, c2=c2f, tau_p=tau, tau_u=tau).assemble())
    z = dt * lam
    R = sum(float(g) * z ** k for k, g in enumerate(stability_polynomial_coeffs()))
    assert np.max(np.abs(R)) <= 1.0 + 1e-12
    # and the bound is not vacuous: twice the step leaves the region
    z2 = 2 * z
    R2 = sum(float(g) * z2 ** k for k, g in enumerate(stability_polynomial_coeffs()))
    assert np.max(np.abs(R2)) > 1.0
