"""Pin: the oracle's time stepper on a method-of-lines system against exact
Fourier-mode decay (1D periodic heat equation, 64-point central differences,
T = 0.1, 16 slices x 25 steps, 8 seeded modes).

Each Fourier mode k of the discrete Laplacian has eigenvalue
lambda_k = -(4/h^2) sin^2(pi k h); one LSRK step multiplies its amplitude by
R(dt lambda_k), and the continuous solution decays as exp(-4 pi^2 k^2 t).
"""

import numpy as np

from oracle.heat import heat_rhs, heat_integrate, heat_eigenvalues
from oracle.lsrk import stability_polynomial_coeffs
from workloads import make_heat_problem


def _mode_amplitudes(y, kmax):
    n = len(y)
    c = np.fft.rfft(y) / (n / 2)
    return c[1:kmax + 1]


def test_eigenvalues_of_difference_operator():
    n = 64
    lam = heat_eigenvalues(n)
    x = np.arange(n) / n
    for k in (1, 5, 13):
        y = np.sin(2 * np.pi * k * x + 0.3)
        assert np.max(np.abs(heat_rhs(y, 1.0 / n) - lam[k] * y)) < 1e-9 * abs(lam[k])


def test_fourier_modes_follow_stability_polynomial():
    prob = make_heat_problem()
    y0, dt, n = prob["y0"], prob["dt"], prob["slices"] * prob["steps_per_slice"]
    lam = heat_eigenvalues(prob["n"])
    g = [float(x) for x in stability_polynomial_coeffs()]
    R = lambda z: sum(gk * z ** k for k, gk in enumerate(g))  # noqa: E731
    yT = heat_integrate(y0, dt, n)
    a0 = _mode_amplitudes(y0, 8)
    aT = _mode_amplitudes(yT, 8)
    want = np.array([a0[k - 1] * R(dt * lam[k]) ** n for k in range(1, 9)])
    assert np.max(np.abs(aT - want)) <= 1e-13 * np.max(np.abs(a0))


def test_slices_compose():
    """Sixteen slices of 25 steps equal one sweep of 400 steps (bitwise)."""
    prob = make_heat_problem()
    y = prob["y0"]
    for _ in range(prob["slices"]):
        y = heat_integrate(y, prob["dt"], prob["steps_per_slice"])
    ref = heat_integrate(prob["y0"], prob["dt"], prob["slices"] * prob["steps_per_slice"])
    assert np.array_equal(y, ref)


def test_matches_continuous_decay_to_spatial_order():
    """Against exp(-4 pi^2 k^2 T): the relative error of mode k is the
    second-order spatial error, 4 pi^2 k^2 T (pi k h)^2 / 3 to leading order."""
    prob = make_heat_problem()
    n, T = prob["n"], prob["T"]
    h = 1.0 / n
    yT = heat_integrate(prob["y0"], prob["dt"], prob["slices"] * prob["steps_per_slice"])
    a0 = _mode_amplitudes(prob["y0"], 8)
    aT = _mode_amplitudes(yT, 8)
    for k in (1, 2, 3):
        exact = a0[k - 1] * np.exp(-4 * np.pi ** 2 * k ** 2 * T)
        rel = abs(aT[k - 1] / exact - 1.0)
        lead = 4 * np.pi ** 2 * k ** 2 * T * (np.pi * k * h) ** 2 / 3
        assert rel < 1.5 * lead + 1e-12
        assert rel > 0.5 * lead
