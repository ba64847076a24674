"""ctypes declarations of the C ABI in include/ptsolve.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libptsolve.so")

PT_OK = 0
PT_ERR_INVALID = -1
PT_ERR_HIP = -3
PT_ERR_NOT_CONVERGED = -4
PT_ERR_BREAKDOWN = -5
PT_ERR_NONFINITE = -6
PT_ERR_DIVERGED = -7
PT_ERR_WORKSPACE = -8

PT_FP64 = 0
PT_FP32_REFINE = 1
PT_INNER_GALERKIN1 = 0
PT_INNER_COCG = 1
PT_VC_DEFAULT = 0
PT_VC_V11 = 1
PT_VC_V01 = 2
PT_WAVE_SIN = 0
PT_WAVE_COS = 1
PT_NU_RATIONAL = 0
PT_NU_EXPCAP = 1


class Rect(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("x1", C.c_double), ("y1", C.c_double)]


class Region(C.Structure):
    _fields_ = [("sigma", C.c_double), ("a", C.c_double), ("b", C.c_double), ("c", C.c_double),
                ("d", C.c_double), ("j", C.c_double), ("nu_hat", C.c_double)]


class Problem(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("N", C.c_int32), ("T", C.c_double),
        ("sigma_in", C.c_double), ("sigma_rect", Rect),
        ("nu_a", C.c_double), ("nu_b", C.c_double), ("nu_out", C.c_double), ("nu_rect", Rect),
        ("J0", C.c_double), ("coil_rect", Rect), ("waveform", C.c_int32),
        ("nu_max", C.c_double),
        ("d_theta", C.c_void_p), ("d_sigma", C.c_void_p), ("d_load", C.c_void_p),
        ("law", C.c_int32), ("nregions", C.c_int32), ("d_region", C.c_void_p), ("regions", C.POINTER(Region)),
    ]


class Options(C.Structure):
    _fields_ = [
        ("tol", C.c_double), ("max_outer", C.c_int32), ("check_every", C.c_int32),
        ("precision", C.c_int32), ("inner", C.c_int32), ("inner_iters", C.c_int32),
        ("vc_sweeps", C.c_int32), ("vc_omega", C.c_double), ("use_initial_guess", C.c_int32),
        ("diverge_factor", C.c_double), ("xcd_remap", C.c_int32), ("timing", C.c_int32),
        ("grid_slot", C.c_int32), ("grid_team", C.c_int32), ("adjoint", C.c_int32),
        ("init_static", C.c_int32), ("init_tol", C.c_double), ("stop_relative_initial", C.c_int32),
        ("krylov_dim", C.c_int32), ("forcing", C.c_double), ("max_krylov", C.c_int32),
        ("graph", C.c_int32), ("inner_rtol", C.c_double), ("breakdown_tol", C.c_double),
        ("vc_cycle", C.c_int32), ("timing_mask", C.c_int32),
        ("grid_restrict", C.c_int32), ("grid_up", C.c_int32), ("grid_matvec", C.c_int32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("outer_iters", C.c_int32), ("rel_residual", C.c_double), ("f_norm", C.c_double),
        ("time_ms", C.c_double), ("residual_history", C.POINTER(C.c_double)),
        ("history_cap", C.c_int32), ("history_len", C.c_int32),
        ("kernel_ms", C.POINTER(C.c_double)), ("kernel_launches", C.POINTER(C.c_int64)),
        ("converged_at", C.c_int32), ("init_iters", C.c_int32), ("rel_initial", C.c_double),
        ("krylov_iters", C.c_int32), ("inner_iters_max", C.c_int32), ("inner_iters_sum", C.c_int64),
    ]


PT_KERNEL_CLASSES = 15


_lib = None


def load():
    """Load the in-tree HIP library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2502_21013_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, sz, i32, dp = C.c_void_p, C.c_size_t, C.c_int32, C.POINTER(C.c_double)
    pplan = C.POINTER(C.c_void_p)
    sig = {
        "pt_options_default": (None, [C.POINTER(Options)]),
        "pt_plan_create": (i32, [C.POINTER(Problem), C.POINTER(Options), pplan]),
        "pt_plan_destroy": (None, [vp]),
        "pt_plan_workspace_bytes": (i32, [vp, C.POINTER(C.c_size_t)]),
        "pt_plan_check_bounds": (i32, [vp, C.c_char_p, sz]),
        "pt_solve": (i32, [vp, vp, sz, vp, vp, C.POINTER(Stats)]),
        "pt_solve_noalloc": (i32, [vp, vp, vp, C.POINTER(Stats)]),
        "pt_plan_create_batch": (i32, [C.POINTER(Problem), i32, C.POINTER(Options), pplan]),
        "pt_plan_batch_size": (i32, [vp, C.POINTER(C.c_int32)]),
        "pt_solve_batch": (i32, [vp, vp, sz, vp, vp, C.POINTER(Stats)]),
        "pt_solve_many": (i32, [i32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_size_t),
                                C.POINTER(C.c_void_p), C.POINTER(C.POINTER(Stats)), C.POINTER(C.c_int32),
                                C.POINTER(C.c_void_p), i32]),
        "pt_residual": (i32, [vp, vp, sz, vp, vp, vp, dp, dp]),
        "pt_residual_spectrum": (i32, [vp, vp, sz, vp, vp, vp, dp, dp]),
        "pt_apply_K": (i32, [vp, vp, sz, vp, vp, i32, vp]),
        "pt_time_rfft": (i32, [vp, vp, sz, vp, vp, vp]),
        "pt_device_reciprocals": (i32, [vp, vp, C.c_int64, vp]),
        "pt_time_irfft": (i32, [vp, vp, sz, vp, vp, vp]),
        "pt_shifted_apply": (i32, [vp, vp, sz, vp, vp, vp]),
        "pt_precond_apply": (i32, [vp, vp, sz, vp, vp, vp]),
        "pt_periodic_solve": (i32, [vp, vp, sz, vp, vp, i32, vp]),
        "pt_adjoint_solve": (i32, [vp, vp, sz, vp, vp, vp, C.POINTER(Stats)]),
        "pt_loss_gradients": (i32, [vp, vp, sz, vp, vp, vp, vp, i32, dp, vp]),
        "pt_newton_solve": (i32, [vp, vp, sz, vp, vp, C.POINTER(Stats)]),
        "pt_jacobian_apply": (i32, [vp, vp, sz, vp, vp, vp, i32, vp]),
        "pt_status_string": (C.c_char_p, [i32]),
        "pt_last_error": (C.c_char_p, []),
        "pt_version": (i32, []),
        "pt_kernel_class_name": (C.c_char_p, [i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
