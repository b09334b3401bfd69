"""MI355X-native sparsifying-preconditioner solver (Ying, arXiv:1409.0297).

The compute path lives in the HIP library ``libspp.so`` (C ABI declared in
``include/spp.h``); this package only marshals arguments to it.  Importing
the package does not touch the GPU; the library is loaded on first use and
a missing build raises immediately -- there is no fallback path.
"""
from .binding import (SPP_C128, SPP_C64_FRONTS, SPP_EBREAKDOWN, SPP_EHIP, SPP_EINVAL,  # noqa: F401
                      SPP_ENOMEM, SPP_ENOTIMPL, SPP_ESINGULAR_SHIFT, SPP_HELMHOLTZ, SPP_MAXWELL,
                      SPP_NOT_CONVERGED, SPP_OK, SPP_ORDER_BISECT, SPP_ORDER_OCTREE,
                      SPP_SCHRODINGER, SPP_F_UNPRECONDITIONED, SPP_F_TIMING, SPP_F_PARTIAL_PIVOTING, SPP_F_GRAPHS, SPP_F_PERSISTENT, SPP_F_AUTOTUNE, KERNEL_CLASSES, SppError, Solver, BatchSolver, library,
                      library_path, spp_apply_green, spp_apply_operator, spp_apply_precond,
                      spp_apply_q, spp_destroy, spp_error_string, spp_get_coefficients,
                      spp_get_stencil, spp_kernel_timing, spp_kernel_timing_reset, spp_last_error,
                      spp_setup, spp_setup_batch, spp_get_shift, spp_solve, spp_stats,
                      CNN, CnnError, SPP_CNN_BF16, SPP_CNN_F32, spp_attach_cnn, spp_learned_stats,
                      spp_get_krylov, spp_autotune, spp_solve_batch, TorchAllocator)
