"""MI355X symmetric interior-penalty DG elliptic solver.

The compute path is libipdg.so (HIP kernels for gfx950 behind the C ABI in
include/ipdg.h); this package is its Python binding.
"""
from .ipdg import (Mesh, SolveOpts, SolveInfo, IpdgError, default_opts, lib, solve_batch,  # noqa: F401
                   mesh_check, reference_element, ax_variant, set_ax_variant, probe_copy, probe_fma, F64, F32, PC_NONE, PC_JACOBI, PC_BLOCK_MASS,
                   PC_PMG, PREC_FP64, PREC_MIXED, PREC_FP32_OPERATOR, BC_INTERIOR, BC_DIRICHLET, BC_NEUMANN)
