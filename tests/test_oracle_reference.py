"""Pins for the oracle's reference-element building blocks: Gauss and
Gauss-Lobatto points against closed forms and against an independent root
finder, quadrature exactness, orthonormality, and derivative / face
evaluation against exact polynomial calculus."""

import numpy as np
import pytest

from oracle.basis import gauss_legendre, gll_nodes, ReferenceQuad
from workloads import gll_points


def test_gll_closed_forms():
    assert np.allclose(gll_nodes(1), [-1, 1], atol=0, rtol=0)
    assert np.allclose(gll_nodes(2), [-1, 0, 1], atol=1e-16)
    s = 1 / np.sqrt(5)
    assert np.allclose(gll_nodes(3), [-1, -s, s, 1], atol=2e-16)
    s = np.sqrt(3 / 7)
    assert np.allclose(gll_nodes(4), [-1, -s, 0, s, 1], atol=2e-16)


@pytest.mark.parametrize("N", range(1, 9))
def test_gll_newton_matches_polynomial_roots(N):
    # oracle: Newton on P_N'; inputs: numpy companion-matrix roots of P_N'
    assert np.max(np.abs(gll_nodes(N) - gll_points(N))) < 5e-15


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_gauss_exactness(n):
    x, w = gauss_legendre(n)
    for m in range(2 * n):
        exact = (1 - (-1) ** (m + 1)) / (m + 1)
        assert abs(np.dot(w, x ** m) - exact) < 1e-14
    m = 2 * n
    assert abs(np.dot(w, x ** m) - 2 / (m + 1)) > 1e-6


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_orthonormal_mass(N):
    ref = ReferenceQuad(N, N + 2)
    assert np.max(np.abs(ref.Mhat - np.eye(ref.Np))) < 1e-14


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_derivatives_and_faces_of_monomials(N):
    ref = ReferenceQuad(N, N + 2)
    g = ref.gll
    rn = np.tile(g, N + 1)
    sn = np.repeat(g, N + 1)
    for i in range(N + 1):
        for j in range(N + 1):
            nodal = rn ** i * sn ** j
            c = np.linalg.solve(ref.Vn, nodal)
            r, s = ref.rq, ref.sq
            assert np.allclose(ref.V @ c, r ** i * s ** j, atol=1e-13)
            dr = i * r ** max(i - 1, 0) * s ** j
            ds = j * r ** i * s ** max(j - 1, 0)
            assert np.allclose(ref.Vr @ c, dr, atol=1e-12)
            assert np.allclose(ref.Vs @ c, ds, atol=1e-12)
            for f, (fr, fs) in enumerate(ref.face_rs):
                assert np.allclose(ref.Vf[f] @ c, fr ** i * fs ** j, atol=1e-13)
