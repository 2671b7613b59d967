"""CPU oracle for the WADG acoustic sweep -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 NumPy implementation of what the GPU path computes,
written from the paper (Chan, Hewett, Warburton, "Weight-adjusted
discontinuous Galerkin methods: curvilinear meshes"):

* ``basis``   -- orthonormal Legendre modal basis on the reference square,
                 Gauss and Gauss-Lobatto-Legendre points (Section 2).
* ``wadg``    -- strong-weak DG right-hand side on curvilinear quads
                 (Section 4.1), the weight-adjusted mass inverse
                 M_J^{-1} ~ Mhat^{-1} M_{1/J} Mhat^{-1} (Section 4, eq. for
                 the WADG inverse; Section 6.2; Section 7 for c^2), the exact
                 curvilinear-DG mass inverse as a comparator, L2 errors,
                 the weight-adjusted energy.
* ``lsrk``    -- low-storage five-stage fourth-order Runge-Kutta (the
                 paper's time integrator, Section 5.2, Carpenter-Kennedy).
* ``heat``    -- 1D periodic heat equation by second-order differences, a
                 method-of-lines system whose Fourier modes have closed forms.
* ``parareal``-- serial-reference parareal iteration over time slices.
* ``adjoint`` -- gradient of a terminal objective with respect to the start
                 state and a wave-speed scale, by dense transposition and
                 tangent-linear sensitivity (small meshes).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path:
it uses a modal basis and explicit per-element matrices where the GPU uses a
nodal basis and sum-factorised tensor contractions.  Its only common
dependency is ``workloads`` (seeded inputs, no discretisation arithmetic).

Parity status: every function is pinned by a test under ``tests/`` against
closed forms, invariants or statements of the paper (see test docstrings);
none is marked "parity unpinned".
"""

from .basis import (gauss_legendre, gll_nodes, legendre_orthonormal,  # noqa: F401
                    ReferenceQuad)
from .lsrk import LSRK54, lsrk_integrate, stability_polynomial_coeffs  # noqa: F401
from .wadg import WADGOracle  # noqa: F401
from .heat import heat_rhs, heat_integrate, heat_eigenvalues  # noqa: F401
from .parareal import parareal, wadg_propagators  # noqa: F401
from .adjoint import TerminalObjective, step_matrix, step_matrix_derivative  # noqa: F401
