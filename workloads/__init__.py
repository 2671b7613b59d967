"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This package builds *inputs only*: periodic curvilinear quadrilateral meshes
(node coordinates at Gauss-Lobatto-Legendre points plus face connectivity),
initial states, wavespeed fields and closed-form exact solutions of the
acoustic system.  It contains none of the discretisation's arithmetic (no
quadrature, no metric terms, no fluxes, no mass matrices, no time stepping):
the oracle and the HIP library each compute those on their own from these
arrays.

State layout used everywhere on the boundary: ``Q[s][f][n][k]`` -- slice ``s``,
field ``f`` in (p, u, v), local node ``n = a + (N+1) b`` (``a`` along the
reference r direction, ``b`` along s), element ``k`` fastest.
"""

from .mesh import gll_points, periodic_quad_mesh, periodic_cover, QuadMesh  # noqa: F401
from .fields import (  # noqa: F401
    wave_modes, PlaneWaveSolution, smooth_pressure, uniform_pressure,
    c2_constant, c2_layered, pack_state, unpack_state, heat_initial,
)
from .configs import (CONFIGS, SENSITIVITY, make_problem, make_heat_problem,  # noqa: F401
                      make_sensitivity_problem, SensitivityProblem, BATCHES, BatchMember,
                      batch_shapes, make_batch)
