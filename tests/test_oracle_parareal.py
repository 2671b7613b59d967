"""Pins for the oracle's parareal iteration against properties that hold by
construction of the method (the statements about when the parallel iterate
reproduces the serial fine solution):

* after k iterations, slices 0..k equal the serial fine sweep (to rounding);
* after S iterations the whole iterate equals the serial fine sweep;
* with G = F the first iteration is already exact;
* on a scalar linear problem the iterate matches the closed form of the
  parareal error recursion.
"""

import numpy as np
import pytest

from oracle import WADGOracle
from oracle.parareal import parareal, wadg_propagators
from workloads import make_problem


@pytest.fixture(scope="module")
def setup():
    prob = make_problem("wadg4", slices=[0])
    o = WADGOracle(prob.mesh, nq1=prob.nq1, c2=prob.c2)
    F, G = wadg_propagators(o, prob.dt, 4, 1)
    S = 6
    serial = [prob.Q0[0]]
    for _ in range(S):
        serial.append(F(serial[-1]))
    return prob, F, G, S, np.stack(serial)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("k", [1, 2, 4])
def test_first_k_slices_are_exact_after_k_iterations(setup, k):
    prob, F, G, S, serial = setup
    U, it, _ = parareal(F, G, prob.Q0[0], S, max_iter=k, tol=0.0)
    assert it == k
    for s in range(k + 1):
        assert _rel(U[s], serial[s]) < 1e-13
    # and not yet beyond (the coarse propagator is not exact)
    assert _rel(U[S], serial[S]) > 1e-10


def test_S_iterations_reproduce_serial_sweep(setup):
    prob, F, G, S, serial = setup
    U, it, change = parareal(F, G, prob.Q0[0], S, max_iter=S, tol=0.0)
    for s in range(S + 1):
        assert _rel(U[s], serial[s]) < 1e-13


def test_converges_before_S_with_tolerance(setup):
    """The stopping rule (largest relative change <= tol) ends the iteration
    before S, with the iterate within a small multiple of tol of the serial
    sweep (the change lags the error by about one iteration)."""
    prob, F, G, S, serial = setup
    U, it, change = parareal(F, G, prob.Q0[0], S, max_iter=S, tol=1e-6)
    assert change <= 1e-6 and it < S
    assert max(_rel(U[s], serial[s]) for s in range(S + 1)) < 1e-6


def test_exact_coarse_propagator_converges_in_one_iteration(setup):
    prob, F, _, S, serial = setup
    U, it, change = parareal(F, F, prob.Q0[0], S, max_iter=3, tol=1e-14)
    assert it <= 2
    for s in range(S + 1):
        assert _rel(U[s], serial[s]) < 1e-13


def test_scalar_closed_form():
    """y' = lam y, F = exp(lam dT), G = 1 + lam dT: the iterate is a
    polynomial in (F - G) with binomial coefficients:
    U_n^k = sum_{j=0..k} C(n, j) (F - G)^j G^{n-j} y0."""
    from math import comb
    lam, dT, S, y0 = -0.7 + 0.4j, 0.3, 8, 1.0
    Fv, Gv = np.exp(lam * dT), 1 + lam * dT
    F = lambda y: Fv * y   # noqa: E731
    G = lambda y: Gv * y   # noqa: E731
    for k in range(0, 5):
        U, _, _ = parareal(F, G, np.array([y0 + 0j]), S, max_iter=k, tol=-1.0)
        for n in range(S + 1):
            want = sum(comb(n, j) * (Fv - Gv) ** j * Gv ** (n - j) for j in range(min(k, n) + 1))
            assert abs(U[n][0] - want) < 1e-14
