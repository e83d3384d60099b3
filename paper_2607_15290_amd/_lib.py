"""ctypes loader and C structure mirrors of include/llg.h.

Loads the in-tree HIP library ``libllg.so``; raises ImportError when it has
not been built (there is no fallback of any kind).  torch is imported first so
that the library binds to the HIP runtime torch already loaded (one runtime
per process, so torch streams and device pointers are valid in the library).
"""

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library links against)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libllg.so")

c_double_p = ctypes.POINTER(ctypes.c_double)


class LLGParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("cexc", ctypes.c_double), ("dt", ctypes.c_double),
                ("theta", ctypes.c_double), ("shift", ctypes.c_double), ("h_uniform", ctypes.c_double * 3),
                ("h_field", ctypes.c_void_p), ("demag", ctypes.c_double), ("aniso_k", ctypes.c_double),
                ("aniso_axis", ctypes.c_double * 3)]


class LLGSolverOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("maxiter", ctypes.c_int), ("max_outer", ctypes.c_int),
                ("use_x0", ctypes.c_int), ("rtol", ctypes.c_double), ("inner_rtol", ctypes.c_double),
                ("prec", ctypes.c_int), ("precond", ctypes.c_int), ("orth", ctypes.c_int),
                ("picard_norm", ctypes.c_int), ("transpose", ctypes.c_int),
                ("fuse_update", ctypes.c_int)]


class LLGSolverStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("cycles", ctypes.c_int), ("outer_steps", ctypes.c_int),
                ("converged", ctypes.c_int), ("rel_res_true", ctypes.c_double), ("rel_res_prec", ctypes.c_double),
                ("restarts", ctypes.c_int), ("ms", ctypes.c_double)]


class LLGStepStats(ctypes.Structure):
    _fields_ = [("picard_iters", ctypes.c_int), ("lin_iters_total", ctypes.c_int), ("converged", ctypes.c_int),
                ("picard_rel_change", ctypes.c_double), ("max_len_err", ctypes.c_double),
                ("energy_before", ctypes.c_double), ("energy_after", ctypes.c_double),
                ("dissipation_defect", ctypes.c_double), ("inexact_correction", ctypes.c_double),
                ("v_norm2", ctypes.c_double)]


class LLGKernelProfile(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_int), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


# name -> (restype, argtypes); mirrors include/llg.h
P = ctypes.c_void_p
I = ctypes.c_int
SIGNATURES = {
    "llg_ctx_create": (I, [ctypes.POINTER(ctypes.c_void_p), I, I, I, ctypes.c_double, I]),
    "llg_ctx_create_cell": (I, [ctypes.POINTER(ctypes.c_void_p), I, I, I, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, I]),
    "llg_ctx_destroy": (I, [P]),
    "llg_workspace_bytes": (ctypes.c_size_t, [P, I, I]),
    "llg_matvec": (I, [P, ctypes.POINTER(LLGParams), P, P, P, I, P]),
    "fft_hss_apply": (I, [P, ctypes.POINTER(LLGParams), P, P, P, I, P]),
    "llg_matvec_f32": (I, [P, ctypes.POINTER(LLGParams), P, P, P, I, P]),
    "fft_hss_apply_f32": (I, [P, ctypes.POINTER(LLGParams), P, P, P, I, P]),
    "llg_precond_op": (I, [P, ctypes.POINTER(LLGParams), P, P, P, P, I, ctypes.c_longlong, P, P]),
    "llg_precond_op_f32": (I, [P, ctypes.POINTER(LLGParams), P, P, P, P, I, P, I, ctypes.c_longlong, P, P]),
    "gmres_solve": (I, [P, ctypes.POINTER(LLGParams), P, P, P, ctypes.POINTER(LLGSolverOpts),
                        ctypes.POINTER(LLGSolverStats), P, ctypes.c_size_t, P]),
    "gmres_solve_noalloc": (I, [P, ctypes.POINTER(LLGParams), P, P, P, ctypes.POINTER(LLGSolverOpts),
                                ctypes.POINTER(LLGSolverStats), P]),
    "llg_step_euler": (I, [P, ctypes.POINTER(LLGParams), P, P, P, ctypes.POINTER(LLGSolverOpts),
                           ctypes.POINTER(LLGStepStats), P, ctypes.c_size_t, P]),
    "llg_step_midpoint": (I, [P, ctypes.POINTER(LLGParams), P, P, P, ctypes.c_double, I,
                              ctypes.POINTER(LLGSolverOpts), ctypes.POINTER(LLGStepStats), P, ctypes.c_size_t, P]),
    "llg_step_midpoint_adjoint": (I, [P, ctypes.POINTER(LLGParams), P, P, P, P, P, c_double_p,
                                      ctypes.POINTER(LLGSolverOpts), ctypes.POINTER(LLGSolverStats), P,
                                      ctypes.c_size_t, P]),
    "llg_energy": (I, [P, ctypes.POINTER(LLGParams), P, c_double_p, P]),
    "llg_rhs": (I, [P, ctypes.POINTER(LLGParams), P, P, P]),
    "llg_profile_enable": (I, [P, I]),
    "llg_profile_read": (I, [P, ctypes.POINTER(LLGKernelProfile), I]),
    "llg_profile_select": (I, [P, ctypes.c_char_p]),
    "llg_last_error": (ctypes.c_char_p, []),
}

STATUS = {0: "LLG_OK", 1: "LLG_EARG", 2: "LLG_EZERO_M", 3: "LLG_ENOCONV", 4: "LLG_EPICARD", 5: "LLG_ENAN",
          6: "LLG_EHIP", 7: "LLG_ENOMEM", 8: "LLG_EUNSUPPORTED"}

_lib = None


def load():
    """Load libllg.so once; ImportError if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built ({LIB_PATH} missing); run: python -m paper_2607_15290_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
