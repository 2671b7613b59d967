"""MI355X-native weight-adjusted DG (WADG) sweep for the acoustic wave
equation on curvilinear quadrilateral meshes.

``binding`` exposes the C ABI of ``libwadg.so`` under its C names;
``solver.Solver`` wraps it with torch device memory.  Importing the package
fails loudly when the HIP library has not been built.
"""

from . import binding  # noqa: F401  (raises if libwadg.so is missing)
from .binding import (  # noqa: F401
    wadg_quadrature_points, wadg_geometry, wadg_cfl_number, WADG_CFL_MAX, wadg_create,
    wadg_destroy, wadg_state_doubles, wadg_workspace_bytes, wadg_rhs, wadg_integrate,
    wadg_workspace_bytes_fp32, wadg_integrate_fp32, wadg_parareal_workspace_bytes,
    wadg_parareal, wadg_norms_workspace_bytes, wadg_norms, wadg_l2_norms_workspace_bytes,
    wadg_l2_norms, wadg_set_schedule, wadg_set_kernel, wadg_kernel_in_use, WADG_KERNEL_AUTO,
    WADG_KERNEL_STREAMED, WADG_KERNEL_RESIDENT, WADG_KERNEL_SPLIT, WADG_KERNEL_PIPE,
    wadg_set_c2_scale,
    wadg_adjoint_workspace_bytes, wadg_forward_checkpoints, wadg_adjoint, wadg_status_string,
    wadg_last_error, MeshDesc, WadgError, tile_state, untile_state,
)
from .solver import Solver, Batch  # noqa: F401
