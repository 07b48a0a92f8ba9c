"""MI355X (gfx950) OSRC-preconditioned PMCHWT boundary element hot path.

Python face of the C-ABI library ``libbem.so`` (declared in include/bem.h):
mesh state, the matrix-free permuted PMCHWT (and Mueller) Galerkin matvec, the OSRC Pade
preconditioner, plane-wave right-hand sides, the preconditioned GMRES solve,
the far field and the field off the surface.  All arithmetic runs in the library's HIP kernels.
"""
from ._binding import (BEM_FP32, BEM_FP32_DENSE, BEM_FP32_HMAT, BEM_FP64, BEM_FP64_DENSE, BemError, Mesh, Server, SolveInfo,
                       SolveOpts,
                       default_opts, far_field, hmat_info, lib, muller_matvec, osrc_apply, osrc_apply_noalloc, osrc_info,
                       pmchwt_field, pmchwt_matvec, pmchwt_matvec_multi, pmchwt_solve_multi,
                       pmchwt_rhs, pmchwt_solve, profile_enable, profile_read,
                       autotune, tune_cache_load, tune_clear, tune_get, tune_lookup, tune_set,
                       valu_rates)

__all__ = ["BEM_FP32", "BEM_FP32_DENSE", "BEM_FP32_HMAT", "BEM_FP64", "BEM_FP64_DENSE", "BemError", "Mesh", "Server", "SolveInfo",
           "SolveOpts",
           "default_opts", "far_field", "hmat_info", "lib", "muller_matvec", "osrc_apply", "osrc_apply_noalloc", "osrc_info",
           "pmchwt_field",
           "pmchwt_matvec", "pmchwt_matvec_multi", "pmchwt_solve_multi",
           "pmchwt_rhs", "pmchwt_solve", "profile_enable", "profile_read",
           "autotune", "tune_cache_load", "tune_clear", "tune_get", "tune_lookup", "tune_set",
           "valu_rates"]
