"""Pins for the oracle's time integrator (LSRK(5,4), paper Section 5.2).

The coefficients are checked against mathematics, not against a retyped
copy: the Butcher tableau derived from the 2N-storage recursion must satisfy
the eight fourth-order conditions, its abscissae must equal the published
stage times, and the stepper loop must reproduce the stability polynomial
on y' = lambda y and the dense matrix polynomial R(dt L)^n on a linear system.
"""

import os
from fractions import Fraction

import numpy as np
import pytest

from oracle.lsrk import LSRK54, butcher_tableau, stability_polynomial_coeffs, lsrk_integrate, C_RAT


def _load_golden(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "lsrk54_carpenter_kennedy.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t) for t in line.split()]
            rows.append((Fraction(v[1], v[2]), Fraction(v[3], v[4]), Fraction(v[5], v[6])))
    return rows


def test_coefficients_match_published_table(golden_dir):
    rows = _load_golden(golden_dir)
    for i, (a, b, c) in enumerate(rows):
        assert LSRK54.A[i] == float(a)
        assert LSRK54.B[i] == float(b)
        assert LSRK54.C[i] == float(c)


def test_fourth_order_conditions():
    a, b, c = butcher_tableau(exact=True)
    s = 5
    one = [Fraction(1)] * s

    def dot(x, y):
        return sum(xi * yi for xi, yi in zip(x, y))

    def mat(A, x):
        return [dot(row, x) for row in A]

    c2 = [ci * ci for ci in c]
    c3 = [ci ** 3 for ci in c]
    Ac = mat(a, c)
    conds = {
        "b.1 = 1": (dot(b, one), Fraction(1)),
        "b.c = 1/2": (dot(b, c), Fraction(1, 2)),
        "b.c^2 = 1/3": (dot(b, c2), Fraction(1, 3)),
        "b.Ac = 1/6": (dot(b, Ac), Fraction(1, 6)),
        "b.c^3 = 1/4": (dot(b, c3), Fraction(1, 4)),
        "b.(c*Ac) = 1/8": (dot(b, [ci * x for ci, x in zip(c, Ac)]), Fraction(1, 8)),
        "b.Ac^2 = 1/12": (dot(b, mat(a, c2)), Fraction(1, 12)),
        "b.AAc = 1/24": (dot(b, mat(a, Ac)), Fraction(1, 24)),
    }
    for name, (got, want) in conds.items():
        assert abs(float(got - want)) < 1e-15, name


def test_abscissae_equal_published_stage_times():
    _, _, c = butcher_tableau(exact=True)
    for ci, Ci in zip(c, C_RAT):
        assert abs(float(ci - Ci)) < 1e-15


def test_stability_polynomial():
    g = stability_polynomial_coeffs()
    want = [1, 1, 1 / 2, 1 / 6, 1 / 24]
    for k in range(5):
        assert abs(float(g[k]) - want[k]) < 1e-15
    # fifth-order coefficient of this scheme (a known property: 1/200)
    assert abs(float(g[5]) - 1 / 200) < 1e-12


@pytest.mark.parametrize("z", [-0.5, -2.0, 1j * 1.5, -1.0 + 2.0j, -4.0])
def test_scalar_step_equals_stability_polynomial(z):
    g = [float(x) for x in stability_polynomial_coeffs()]
    R = sum(gk * z ** k for k, gk in enumerate(g))
    n = 7
    y = lsrk_integrate(lambda y: z * y, np.array([1.0 + 0j]), 1.0, n)
    assert abs(y[0] - R ** n) <= 1e-13 * max(1.0, abs(R) ** n)


def test_linear_system_equals_matrix_polynomial():
    rng = np.random.default_rng(0)
    L = rng.standard_normal((12, 12))
    L = L - L.T - 0.3 * np.eye(12)          # dissipative, non-normal-ish
    y0 = rng.standard_normal(12)
    dt, n = 0.05, 9
    g = [float(x) for x in stability_polynomial_coeffs()]
    R = sum(gk * np.linalg.matrix_power(dt * L, k) for k, gk in enumerate(g))
    want = np.linalg.matrix_power(R, n) @ y0
    got = lsrk_integrate(lambda y: L @ y, y0, dt, n)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


def test_stability_bounds_on_axes():
    """R is stable on [-4.65, 0] and on the imaginary axis up to ~3.34."""
    g = [float(x) for x in stability_polynomial_coeffs()]

    def R(z):
        return sum(gk * z ** k for k, gk in enumerate(g))
    assert abs(R(-4.6)) <= 1.0 and abs(R(-4.7)) > 1.0
    assert abs(R(3.3j)) <= 1.0 and abs(R(3.4j)) > 1.0
