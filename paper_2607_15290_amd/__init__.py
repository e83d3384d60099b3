"""MI355X-native FFT-HSS preconditioned GMRES for periodic LLG saddle-point
systems.  The numerical path is the HIP library libllg.so (C ABI in
include/llg.h); this package is its Python binding."""

from .llg import (FP32_IR, FP64, Context, LLGError, Params, fft_hss_apply, fft_hss_apply_f32,  # noqa: F401
                  llg_precond_op, llg_precond_op_f32,
                  gmres_solve, gmres_solve_noalloc, llg_energy, llg_rhs, llg_matvec, llg_matvec_f32, llg_step_euler, llg_step_midpoint,
                  llg_step_midpoint_adjoint, llg_profile_enable, llg_profile_read,
                  llg_profile_select)
from .autograd import LLGMidpoint, midpoint_trajectory  # noqa: F401,E402
