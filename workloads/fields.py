"""Initial states, wavespeed fields and exact solutions (inputs only).

Exact solutions are closed forms of the continuous acoustic system with
rho = 1 (the paper's model problem, Section 4.1)

    (1/c^2) p_t + div u = 0,   u_t + grad p = 0,

on the periodic unit square with constant c^2: a standing plane wave
``p = a cos(k.x + phi) cos(w t)``, ``u = a (k/w) sin(k.x + phi) sin(w t)``
with ``w = c |k|`` solves it, and sums of such waves do too.
"""

import numpy as np

TWO_PI = 2.0 * np.pi


def wave_modes(count):
    """The ``count`` lowest wavevectors (m, n) in Z^2 \\ {0} with m > 0 or
    (m = 0, n > 0), sorted by (m^2 + n^2, m, n)."""
    modes = []
    R = 1
    while True:
        cand = [(m, n) for m in range(0, R + 1) for n in range(-R, R + 1)
                if (m > 0 or (m == 0 and n > 0))]
        cand.sort(key=lambda mn: (mn[0] ** 2 + mn[1] ** 2, mn[0], mn[1]))
        # everything with |k|^2 <= R^2 is complete inside the box of radius R
        done = [mn for mn in cand if mn[0] ** 2 + mn[1] ** 2 <= R * R]
        if len(done) >= count:
            return done[:count]
        R += 1


class PlaneWaveSolution:
    """Sum of standing plane waves, exact for constant c^2 on the torus."""

    def __init__(self, modes, amps, phases, c2=1.0):
        self.modes = np.asarray(modes, dtype=float).reshape(-1, 2)
        self.amps = np.asarray(amps, dtype=float)
        self.phases = np.asarray(phases, dtype=float)
        self.c = float(np.sqrt(c2))

    def __call__(self, x, y, t):
        """(p, u, v) at points (x, y) and time t."""
        p = np.zeros(np.shape(x))
        u = np.zeros(np.shape(x))
        v = np.zeros(np.shape(x))
        for (m, n), a, ph in zip(self.modes, self.amps, self.phases):
            kx, ky = TWO_PI * m, TWO_PI * n
            w = self.c * np.hypot(kx, ky)
            th = kx * x + ky * y + ph
            p += a * np.cos(th) * np.cos(w * t)
            s = a * np.sin(th) * np.sin(w * t) / w
            u += s * kx
            v += s * ky
        return p, u, v


def smooth_pressure(mesh, count, seed, c2=1.0):
    """Sum of the ``count`` lowest standing waves with amplitudes a ~ N(0,1)
    then phases phi ~ U[0, 2 pi) drawn from default_rng(seed) in that order.
    Returns the exact solution object; evaluate it at the mesh nodes for a
    nodal initial state at any time."""
    rng = np.random.default_rng(seed)
    modes = wave_modes(count)
    amps = rng.standard_normal(count)
    phases = rng.uniform(0.0, TWO_PI, count)
    return PlaneWaveSolution(modes, amps, phases, c2=c2)


def uniform_pressure(mesh, seed, lo=-0.1, hi=0.1):
    """Nodal pressure p ~ U[lo, hi] per node ([K][Np], drawn in that order);
    the discontinuous field is an admissible DG state."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=mesh.x.shape)


def c2_constant(value=1.0):
    def c2(x, y):
        return np.full(np.shape(x), float(value))
    c2.description = f"c^2 = {value}"
    return c2


def c2_layered(x, y):
    """Heterogeneous wavespeed 1 + 0.5 sin(2 pi x) sin(4 pi y) (in [0.5, 1.5])."""
    return 1.0 + 0.5 * np.sin(TWO_PI * x) * np.sin(2.0 * TWO_PI * y)


c2_layered.description = "c^2 = 1 + 0.5 sin(2 pi x) sin(4 pi y)"


def pack_state(fields):
    """Per-slice nodal fields -> boundary layout.

    ``fields``: array [S][3][K][Np] (element-major, as meshes are stored).
    Returns a C-contiguous float64 array [S][3][Np][K]."""
    f = np.asarray(fields, dtype=np.float64)
    return np.ascontiguousarray(np.swapaxes(f, -1, -2))


def unpack_state(Q):
    """Boundary layout [S][3][Np][K] -> [S][3][K][Np]."""
    return np.ascontiguousarray(np.swapaxes(np.asarray(Q), -1, -2))


def heat_initial(n, count, seed):
    """1D periodic heat workload: y0 = sum_{k=1..count} a_k sin(2 pi k x + phi_k)
    on the grid x_i = i / n, a ~ N(0,1) then phi ~ U[0, 2 pi) from
    default_rng(seed).  Returns (y0, amps, phases)."""
    rng = np.random.default_rng(seed)
    amps = rng.standard_normal(count)
    phases = rng.uniform(0.0, TWO_PI, count)
    x = np.arange(n) / n
    y0 = np.zeros(n)
    for k in range(1, count + 1):
        y0 += amps[k - 1] * np.sin(TWO_PI * k * x + phases[k - 1])
    return y0, amps, phases
