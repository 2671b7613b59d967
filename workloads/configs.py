"""Named synthetic workloads.

The paper measures on curvilinear tetrahedral sphere meshes that are not
available; these periodic curvilinear quadrilateral workloads stand in for
them with the shapes that matter to the sweep: degree N = 3 (the paper's
central degree), isoparametric curved elements with a Jacobian that varies
inside every element, smooth or heterogeneous c^2, upwind fluxes, LSRK(5,4)
steps at a fixed CFL number, and many independent time slices advanced
together.

  heat64   1D periodic heat equation, 64-point second-order differences,
           T = 0.1, 16 slices x 25 steps, 8 seeded Fourier modes (seed 1).
  wadg4    2D acoustic WADG, 4x4 elements, N=3, eps=0.05, c^2=1, tau=1,
           T=0.1 over S=16 slices, 1 step per slice (dt = 6.25e-3), 8 modes
           (seed 1); slice s starts from the exact solution at t_s.
  wadg64   64x64 elements (256x256 nodes per field), N=3, eps=0.05, c^2=1,
           tau=1, T=1 over S=64 slices of 32 steps (dt = 1/2048), 32 modes
           (seed 2); slice s starts from the exact solution at t_s.
  wadg128  128x128 elements (512x512 nodes per field), N=3, eps=0.05,
           c^2 = 1 + 0.5 sin(2 pi x) sin(4 pi y), tau=1, S=256 slices of 10
           steps (dt = 0.5/256/10); slice s starts from nodal p ~ U[-0.1,0.1]
           with seed 3+s and u = 0.
  adj128   sensitivity problem: one trajectory on 128x128 elements, N=3,
           eps=0.05, c^2 = gamma (1 + 0.5 sin(2 pi x) sin(4 pi y)), gamma = 1,
           tau=1, T=0.25 over S=128 checkpointed slices of 10 steps
           (dt = 0.25/1280); start state p0 = 32 modes (seed 5), u = 0;
           target p = 32 modes (seed 6); objective sum over nodes (p(T) -
           p_target)^2.
  adj4     the same on 4x4 elements, S=3 slices of 2 steps (dt = 0.01),
           8 modes (seeds 5 and 6), gamma = 1.3 (oracle-sized).
  batch1000  1000 independent acoustic problems, N=3, eps=0.05, c^2=1,
           tau=1: nodes per field n ~ log-uniform[64, 4096] -> K1D =
           clip(round(sqrt(n)/4), 2, 16); S ~ U{8..128} slices of 4 steps,
           dt = 0.025/K1D (CFL 0.4); p = 4 lowest standing waves with
           a ~ N(0,1), phi ~ U[0, 2 pi) from the problem's spawned generator;
           slice s starts from the exact solution at t = 4 s dt.  Draw order
           from default_rng(4): all n, then all S, then one spawned child
           per problem.
"""

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from .mesh import periodic_quad_mesh, QuadMesh
from .fields import (smooth_pressure, uniform_pressure, c2_constant, c2_layered,
                     pack_state, heat_initial, wave_modes, PlaneWaveSolution)


CONFIGS = {
    "heat64": dict(kind="heat", n=64, T=0.1, slices=16, steps_per_slice=25, modes=8, seed=1),
    "wadg4": dict(kind="wadg", K1D=4, N=3, eps=0.05, c2="const", tau=1.0, T=0.1,
                  S=16, steps_per_slice=1, modes=8, seed=1, init="exact"),
    "wadg64": dict(kind="wadg", K1D=64, N=3, eps=0.05, c2="const", tau=1.0, T=1.0,
                   S=64, steps_per_slice=32, modes=32, seed=2, init="exact"),
    "wadg128": dict(kind="wadg", K1D=128, N=3, eps=0.05, c2="layered", tau=1.0, T=0.5,
                    S=256, steps_per_slice=10, seed=3, init="uniform"),
}


SENSITIVITY = {
    "adj128": dict(K1D=128, N=3, eps=0.05, tau=1.0, gamma=1.0, T=0.25, S=128,
                   steps_per_slice=10, modes=32, seed_p0=5, seed_target=6),
    "adj4": dict(K1D=4, N=3, eps=0.05, tau=1.0, gamma=1.3, T=0.06, S=3,
                 steps_per_slice=2, modes=8, seed_p0=5, seed_target=6),
}


@dataclass
class SensitivityProblem:
    name: str
    mesh: QuadMesh
    c0: Callable                # base c^2; the sweep uses gamma * c0
    gamma: float
    tau_p: float
    tau_u: float
    nq1: int
    S: int                      # checkpointed slices of one trajectory
    nsteps: int                 # steps per slice
    dt: float
    y0: np.ndarray              # [3][Np][K] start state
    p_target: np.ndarray        # [Np][K]

    @property
    def N(self):
        return self.mesh.N

    @property
    def K(self):
        return self.mesh.K


def make_sensitivity_problem(name, **overrides):
    cfg = dict(SENSITIVITY[name])
    cfg.update(overrides)
    N, K1D = cfg["N"], cfg["K1D"]
    mesh = periodic_quad_mesh(K1D, N, eps=cfg["eps"])
    Np = (N + 1) ** 2
    p0, _, _ = smooth_pressure(mesh, cfg["modes"], cfg["seed_p0"])(mesh.x, mesh.y, 0.0)
    pt, _, _ = smooth_pressure(mesh, cfg["modes"], cfg["seed_target"])(mesh.x, mesh.y, 0.0)
    fields = np.zeros((1, 3, mesh.K, Np))
    fields[0, 0] = p0
    y0 = pack_state(fields)[0]
    nsteps = cfg["steps_per_slice"]
    return SensitivityProblem(name=name, mesh=mesh, c0=c2_layered, gamma=cfg["gamma"],
                              tau_p=cfg["tau"], tau_u=cfg["tau"], nq1=N + 2, S=cfg["S"],
                              nsteps=nsteps, dt=cfg["T"] / (cfg["S"] * nsteps), y0=y0,
                              p_target=np.ascontiguousarray(pt.T))


@dataclass
class Problem:
    name: str
    mesh: QuadMesh
    c2: Callable
    tau_p: float
    tau_u: float
    nq1: int
    S: int
    dt: float
    nsteps: int                 # steps per slice
    slices: np.ndarray          # which slice indices Q0 holds
    Q0: np.ndarray              # [len(slices)][3][Np][K] float64 start states
    exact: Optional[object] = None
    t_starts: Optional[np.ndarray] = None
    params: dict = field(default_factory=dict)

    @property
    def N(self):
        return self.mesh.N

    @property
    def K(self):
        return self.mesh.K


def make_problem(name, slices=None, nq1=None, **overrides):
    """Build workload ``name`` (see module docstring).  ``slices`` selects a
    subset of slice start states (default: all).  ``overrides`` replace config
    entries (e.g. K1D, S, N, eps) for reduced variants used by tests."""
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    if cfg["kind"] != "wadg":
        raise ValueError(f"{name} is not a WADG workload")
    N, K1D = cfg["N"], cfg["K1D"]
    mesh = periodic_quad_mesh(K1D, N, eps=cfg["eps"], rotate_seed=cfg.get("rotate_seed"))
    c2 = c2_constant(1.0) if cfg["c2"] == "const" else c2_layered
    S = cfg["S"]
    dT = cfg["T"] / S
    nsteps = cfg["steps_per_slice"]
    dt = dT / nsteps
    sl = np.arange(S) if slices is None else np.asarray(slices, dtype=np.int64)
    Np = (N + 1) ** 2
    fields = np.zeros((len(sl), 3, mesh.K, Np))
    exact = None
    t_starts = sl * dT
    if cfg["init"] == "exact":
        exact = smooth_pressure(mesh, cfg["modes"], cfg["seed"])
        for i, t in enumerate(t_starts):
            p, u, v = exact(mesh.x, mesh.y, t)
            fields[i, 0], fields[i, 1], fields[i, 2] = p, u, v
    elif cfg["init"] == "uniform":
        for i, s in enumerate(sl):
            fields[i, 0] = uniform_pressure(mesh, cfg["seed"] + int(s))
    else:
        raise ValueError(cfg["init"])
    return Problem(name=name, mesh=mesh, c2=c2, tau_p=cfg["tau"], tau_u=cfg["tau"],
                   nq1=(N + 2) if nq1 is None else nq1, S=S, dt=dt, nsteps=nsteps,
                   slices=sl, Q0=pack_state(fields), exact=exact, t_starts=t_starts,
                   params=cfg)


def make_heat_problem(name="heat64"):
    cfg = CONFIGS[name]
    y0, amps, phases = heat_initial(cfg["n"], cfg["modes"], cfg["seed"])
    total_steps = cfg["slices"] * cfg["steps_per_slice"]
    return dict(y0=y0, amps=amps, phases=phases, n=cfg["n"], T=cfg["T"],
                slices=cfg["slices"], steps_per_slice=cfg["steps_per_slice"],
                dt=cfg["T"] / total_steps)


BATCHES = {
    "batch1000": dict(count=1000, N=3, eps=0.05, tau=1.0, nodes=(64, 4096), K1D=(2, 16),
                      S=(8, 128), steps_per_slice=4, modes=4, cfl=0.4, seed=4),
}


@dataclass
class BatchMember:
    mesh: QuadMesh
    S: int
    dt: float
    nsteps: int
    Q0: np.ndarray              # [S][3][Np][K] start states
    exact: object


def batch_shapes(name="batch1000", count=None):
    """(K1D, S) of every problem of the batch, without building anything."""
    cfg = BATCHES[name]
    n = cfg["count"] if count is None else count
    rng = np.random.default_rng(cfg["seed"])
    lo, hi = np.log(cfg["nodes"][0]), np.log(cfg["nodes"][1])
    nodes = np.exp(rng.uniform(lo, hi, cfg["count"]))
    S = rng.integers(cfg["S"][0], cfg["S"][1] + 1, cfg["count"])
    k1d = np.clip(np.round(np.sqrt(nodes) / 4.0), cfg["K1D"][0], cfg["K1D"][1]).astype(int)
    return k1d[:n], S[:n], rng


def make_batch(name="batch1000", count=None, members=None):
    """Build the batch (or its first ``count`` problems, or the problems with
    the indices in ``members``).  Every problem draws from its own spawned
    generator, so a subset is identical to the same problems of the full
    batch."""
    cfg = BATCHES[name]
    k1d, S, rng = batch_shapes(name)
    children = rng.spawn(cfg["count"])
    idx = range(cfg["count"] if count is None else count) if members is None else members
    out = []
    for i in idx:
        mesh = periodic_quad_mesh(int(k1d[i]), cfg["N"], eps=cfg["eps"])
        r = children[i]
        modes = wave_modes(cfg["modes"])
        amps = r.standard_normal(cfg["modes"])
        phases = r.uniform(0.0, 2.0 * np.pi, cfg["modes"])
        exact = PlaneWaveSolution(modes, amps, phases)
        dt = cfg["cfl"] / ((cfg["N"] + 1) ** 2 * int(k1d[i]))
        nsteps = cfg["steps_per_slice"]
        fields = np.zeros((int(S[i]), 3, mesh.K, (cfg["N"] + 1) ** 2))
        for s in range(int(S[i])):
            fields[s] = np.stack(exact(mesh.x, mesh.y, s * nsteps * dt))
        out.append(BatchMember(mesh=mesh, S=int(S[i]), dt=dt, nsteps=nsteps,
                               Q0=pack_state(fields), exact=exact))
    return out
