"""MI355X (gfx950) implementation of the parallel-in-time multigrid
preconditioned FGMRES solve for augmented systems (arXiv 2405.04808).

The solver lives in libpitmg.so (HIP kernels behind a C ABI, see
include/pitmg.h); this package holds its sources, its build script and a
thin ctypes binding.
"""
from .pitmg import (Solver, Net, Burgers, solve_batch, PitmgError, default_options, load_library, header_functions,
                    pitmg_options, pitmg_problem, pitmg_stats, LIB_PATH, PROFILE_CLASSES,
                    PITMG_OK, PITMG_NOT_CONVERGED, PITMG_ERR_INVALID, PITMG_ERR_SINGULAR,
                    PITMG_ERR_NONFINITE, PITMG_ERR_HIP, PITMG_ERR_OOM, PITMG_ERR_UNSUPPORTED)

__all__ = ["Solver", "Net", "Burgers", "solve_batch", "PitmgError", "default_options", "load_library", "header_functions",
           "pitmg_options", "pitmg_problem", "pitmg_stats", "LIB_PATH", "PROFILE_CLASSES",
           "PITMG_OK", "PITMG_NOT_CONVERGED", "PITMG_ERR_INVALID", "PITMG_ERR_SINGULAR",
           "PITMG_ERR_NONFINITE", "PITMG_ERR_HIP", "PITMG_ERR_OOM", "PITMG_ERR_UNSUPPORTED"]
