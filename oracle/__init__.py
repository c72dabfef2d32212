"""Plain FP64 CPU oracle for the AMR face transfer of Stokes, Weinzierl, Zhang and
Li, "Fast Higher-Order Interpolation and Restriction in ExaHyPE Avoiding
Non-physical Reflections" (arXiv 2504.15814).

TEST INFRASTRUCTURE ONLY.  This package exists to check the HIP library against
an obviously correct, slow restatement of the method.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
library's product path never does, and it shares no code with the library
(no kernels, headers, helpers, tables or constant generators).

Contents
--------
geometry   face-buffer layout and cell-centre positions (the conventions the
           paper leaves open, stated once)
fit        Taylor terms and the pinned-constant least-squares fit
           (Section 3, "Operator construction"; Appendix C, stencils)
transfer   dense per-subface operators built directly in each physical
           orientation, and their application to batches of faces
           (Section 2, the P / R matrices and their 1/9 segments)
patches    patches with face halos: face views, the same-level halo copy, and
           the transfer composed with them (Section 2)
transfer2d the same transfer in two dimensions (Sections 2-3 are stated for
           any dimension)

Everything is float64 and written for readability, not speed.
"""

from .geometry import (
    face_axes,
    face_extents,
    cell_count,
    cell_index,
    storage_cells,
    coarse_position,
    fine_position,
    coarse_fine_side_half,
    fine_ghost_half,
)
from .fit import taylor_exponents, taylor_term, taylor_stencil, pinned_fit_weights, linear_weights_1d
from .transfer import (
    DLINEAR,
    TAYLOR2,
    TAYLOR3,
    INTERPOLATE,
    RESTRICT,
    interpolation_operator,
    restriction_operator,
    transfer_operator,
    interpolate_faces,
    restrict_faces,
    clear_operator_cache,
)
from . import patches
from . import transfer2d

__all__ = [
    "face_axes",
    "face_extents",
    "cell_count",
    "cell_index",
    "storage_cells",
    "coarse_position",
    "fine_position",
    "coarse_fine_side_half",
    "fine_ghost_half",
    "taylor_exponents",
    "taylor_term",
    "taylor_stencil",
    "pinned_fit_weights",
    "linear_weights_1d",
    "DLINEAR",
    "TAYLOR2",
    "TAYLOR3",
    "INTERPOLATE",
    "RESTRICT",
    "interpolation_operator",
    "restriction_operator",
    "transfer_operator",
    "interpolate_faces",
    "restrict_faces",
    "clear_operator_cache",
    "patches",
    "transfer2d",
]
