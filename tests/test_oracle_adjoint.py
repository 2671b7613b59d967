"""Pins of the oracle's terminal-objective gradient (the discrete adjoint of
the sweep): central finite differences of the oracle's own stepper, the
dot-product identity of the transposed sweep, the linear dependence of the
operator on the wave-speed scale, and agreement of its two routes (dense
transposition with tangent-linear sensitivity vs the reverse 2N-storage
recursion)."""

import numpy as np
import pytest

from workloads import periodic_quad_mesh, c2_layered
from oracle import TerminalObjective, WADGOracle

DT, NSTEPS, GAMMA = 0.01, 4, 1.3


@pytest.fixture(scope="module")
def obj():
    mesh = periodic_quad_mesh(4, 3, eps=0.05, warp="skew", rotate_seed=3)
    return TerminalObjective(mesh, c0=c2_layered)


@pytest.fixture(scope="module")
def data(obj):
    rng = np.random.default_rng(0)
    return rng.standard_normal(obj.shape), rng.standard_normal(obj.shape[1:])


def test_operator_is_linear_in_wave_speed_scale(obj):
    """c^2 enters only the pressure mass inverse, linearly: the operator
    assembled with c^2 = gamma c0^2 equals E(gamma) L_1."""
    o = WADGOracle(obj.o1.mesh, c2=lambda x, y: GAMMA * c2_layered(x, y))
    L = o.assemble()
    assert np.max(np.abs(L - obj.operator(GAMMA))) <= 1e-13 * np.max(np.abs(L))


def test_two_routes_agree(obj, data):
    y0, pt = data
    J1, g1, d1 = obj.gradient(y0, pt, GAMMA, DT, NSTEPS)
    J2, g2, d2 = obj.gradient_reverse(y0, pt, GAMMA, DT, NSTEPS)
    assert abs(J1 - J2) <= 1e-13 * J1
    assert np.max(np.abs(g1 - g2)) <= 1e-13 * np.max(np.abs(g1))
    assert abs(d1 - d2) <= 1e-12 * abs(d1)


def test_objective_equals_stepped_value(obj, data):
    y0, pt = data
    J, _, _ = obj.gradient(y0, pt, GAMMA, DT, NSTEPS)
    assert abs(obj.value(y0, pt, GAMMA, DT, NSTEPS) - J) <= 1e-12 * J


def test_wave_speed_derivative_matches_central_fd(obj, data):
    y0, pt = data
    _, _, dg = obj.gradient(y0, pt, GAMMA, DT, NSTEPS)
    h = 1e-6
    fd = (obj.value(y0, pt, GAMMA + h, DT, NSTEPS)
          - obj.value(y0, pt, GAMMA - h, DT, NSTEPS)) / (2 * h)
    assert abs(fd - dg) <= 1e-7 * abs(dg)


def test_start_state_gradient_matches_central_fd(obj, data):
    """J is quadratic in y0, so central differences are exact up to rounding."""
    y0, pt = data
    J, gy, _ = obj.gradient(y0, pt, GAMMA, DT, NSTEPS)
    rng = np.random.default_rng(7)
    h = 1e-3
    for _ in range(3):
        d = rng.standard_normal(obj.shape)
        d /= np.linalg.norm(d)
        fd = (obj.value(y0 + h * d, pt, GAMMA, DT, NSTEPS)
              - obj.value(y0 - h * d, pt, GAMMA, DT, NSTEPS)) / (2 * h)
        assert abs(fd - np.sum(gy * d)) <= 1e-9 * J


def test_dot_product_identity(obj):
    """<Phi^n x, w> = <x, (Phi^T)^n w>, Phi^n x by the oracle's stepper."""
    rng = np.random.default_rng(11)
    x = rng.standard_normal(obj.shape)
    w = rng.standard_normal(obj.shape)
    o = WADGOracle(obj.o1.mesh, c2=lambda xx, yy: GAMMA * c2_layered(xx, yy))
    lhs = np.sum(o.integrate(x, DT, NSTEPS) * w)
    rhs = np.sum(x * obj.adjoint_apply(w, GAMMA, DT, NSTEPS))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(w)
