"""ctypes declarations of include/fmgeig.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfmgeig.so")

FMG_OK, FMG_PENDING = 0, 1
FMG_EINVAL, FMG_ENOMEM, FMG_ENOCONV, FMG_ENONFINITE, FMG_EHIP = -1, -2, -3, -4, -5
FMG_FP64, FMG_MIXED = 0, 1
FMG_SMOOTH_SGS, FMG_SMOOTH_CG = 0, 1
HISTORY_MAX = 512


class fmg_problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_coarse", C.c_int32), ("n_refine", C.c_int32), ("reserved", C.c_int32),
                ("w_quad", C.c_double * 3), ("w_const", C.c_double), ("zeta", C.c_double),
                ("diffusion", C.c_double * 3)]


class fmg_options(C.Structure):
    _fields_ = [("tol_lambda", C.c_double), ("m", C.c_int32), ("p", C.c_int32), ("nu_pre", C.c_int32),
                ("nu_post", C.c_int32), ("max_final_steps", C.c_int32), ("newton_max_iter", C.c_int32),
                ("newton_tol", C.c_double), ("precision", C.c_int32), ("newton_fixed_iters", C.c_int32),
                ("smoother", C.c_int32), ("reserved", C.c_int32)]


class fmg_tuning(C.Structure):
    _fields_ = [("vpass3d_variant", C.c_int32), ("vpass3d_min_n", C.c_int32), ("vpass2d_wide_min_n", C.c_int32),
                ("vbottom2d_max_n", C.c_int32), ("vpass3d_one_pass", C.c_int32), ("vtile3d", C.c_int32),
                ("reserved", C.c_int32 * 2)]


class fmg_kernel_profile(C.Structure):
    _fields_ = [("launches", C.c_int64), ("seconds", C.c_double), ("bytes", C.c_double), ("units", C.c_double)]


FMG_PROF_VPOST2D_F64, FMG_PROF_VPOST3D_F64, FMG_PROF_VPRE3D_F64, FMG_PROF_MOMENTS3D, FMG_PROF_RHS3D = 1, 2, 3, 4, 5


class fmg_result(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("lambda_rq", C.c_double), ("norm", C.c_double), ("dlambda", C.c_double),
                ("status", C.c_int32), ("levels", C.c_int32), ("steps_total", C.c_int32),
                ("newton_total", C.c_int32), ("seconds", C.c_double), ("wait_seconds", C.c_double),
                ("history_len", C.c_int32),
                ("factor_total", C.c_int32), ("residual", C.c_double), ("gamma_est", C.c_double),
                ("history", C.c_double * HISTORY_MAX)]


P = C.c_void_p
I32 = C.c_int32
I64 = C.c_int64
SZ = C.c_size_t
D = C.c_double

# name -> (restype, argtypes); the exported symbol list the library must provide
SIGNATURES = {
    "fmg_last_error": (C.c_char_p, []),
    "fmg_version": (C.c_char_p, []),
    "fmg_set_fused_vcycle": (C.c_int, [I32]),
    "fmg_get_tuning": (C.c_int, [P]),
    "fmg_set_tuning": (C.c_int, [P]),
    "fmg_autotune_vcycle": (C.c_int, [I32, I32, I32, P, P]),
    "fmg_profile_begin": (C.c_int, [I32, I32]),
    "fmg_profile_end": (C.c_int, [P]),
    "fmg_workspace_bytes": (C.c_int, [P, P, C.POINTER(SZ)]),
    "fmg_solve": (C.c_int, [P, P, P, SZ, P, P, I64, P]),
    "fmg_solve_alloc": (C.c_int, [P, P, P, P, I64, P]),
    "fmg_solve_static": (C.c_int, [P, P, P, P, I64, P]),
    "fmg_footprint_bytes": (SZ, [P, P]),
    "fmg_set_allocator": (C.c_int, [P, P, P]),
    "fmg_batch_solve": (C.c_int, [I32, P, P, P, P, P, P]),
    "fmg_batch_plan_create": (P, [I32, P, P, P]),
    "fmg_batch_plan_run": (C.c_int, [P, P, P, P]),
    "fmg_batch_plan_destroy": (None, [P]),
    "fmg_server_create": (P, [SZ, I32, P]),
    "fmg_server_submit": (C.c_int, [P, P, P, C.POINTER(C.c_uint64)]),
    "fmg_server_poll": (C.c_int, [P, C.c_uint64, P, P, I64]),
    "fmg_server_destroy": (None, [P]),
    "fmg_level_pitch": (I64, [I32, I32]),
    "fmg_level_elems": (I64, [I32, I32]),
    "fmg_pack": (C.c_int, [I32, I32, P, P, P]),
    "fmg_unpack": (C.c_int, [I32, I32, P, P, P]),
    "fmg_op_rhs": (C.c_int, [P, I32, D, P, P, P]),
    "fmg_op_smooth": (C.c_int, [I32, I32, I32, P, P, I32, P]),
    "fmg_op_cg_smooth": (C.c_int, [I32, I32, I32, P, P, I32, P, SZ, P]),
    "fmg_op_residual_restrict": (C.c_int, [I32, I32, I32, P, P, P, P]),
    "fmg_op_prolong": (C.c_int, [I32, I32, I32, P, P, I32, P]),
    "fmg_op_coarse_solve": (C.c_int, [I32, I32, I32, P, P, P]),
    "fmg_op_vcycle": (C.c_int, [I32, I32, I32, I32, I32, P, P, P, SZ, P]),
    "fmg_moments_layout": (C.c_int, [I32, I32, I32, C.POINTER(I32), C.POINTER(SZ)]),
    "fmg_op_moments": (C.c_int, [P, I32, P, P, P, SZ, P]),
    "fmg_op_moments_chunked": (C.c_int, [P, I32, P, P, P, SZ, I32, P]),
    "fmg_small_scratch_bytes": (C.c_int, [I32, I32, C.POINTER(SZ)]),
    "fmg_op_augmented_matrices": (C.c_int, [P, P, P, P, P, P, P, SZ, P]),
    "fmg_op_augmented_solve": (C.c_int, [P, P, P, P, P, SZ, P, C.POINTER(D), C.POINTER(D), C.POINTER(I32),
                                         C.POINTER(I32)]),
    "fmg_op_coarse_nonlinear": (C.c_int, [P, P, P, P, SZ, P, C.POINTER(D), C.POINTER(I32), C.POINTER(I32)]),
    "fmg_op_form_u": (C.c_int, [I32, I32, I32, D, P, P, P, P]),
    "fmg_op_forms": (C.c_int, [P, I32, P, P, P, P]),
}

_lib = None


def load(path: str | None = None):
    """Load libfmgeig.so.  Raises when the HIP library has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libfmgeig.so not found at {p}; build it with `python -m paper_1502_04657_amd.build`")
    lib = C.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib
