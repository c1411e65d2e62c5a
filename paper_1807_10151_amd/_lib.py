"""ctypes declarations of libsuppcg's C ABI (include/suppcg.h).

Argument marshalling only: every computation happens in the HIP library.  If
the library has not been built the import of the binding fails loudly; there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_uint32, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsuppcg.so")

# status codes (suppcg.h)
SP_OK = 0
SP_ERR_ARG = 1
SP_ERR_NOT_SPD = 2
SP_ERR_NONFINITE = 3
SP_ERR_HIP = 4
SP_ERR_ALLOC = 5
SP_MAXITER = 16
SP_CONVERGED = 17
SP_BREAKDOWN_CONVERGED = 18
SP_TRIALS_EXHAUSTED = 19

SP_PRECOND_NONE = 0
SP_PRECOND_RAMP = 1
SP_PRECOND_LEARNED = 2

SP_FLAG_REPLAY = 1
SP_FLAG_GRAPH = 2
SP_FLAG_AUTOTUNE = 4
SP_FLAG_RESUME = 8
SP_FLAG_ASYNC = 16

SP_PROF_PROJECT = 0
SP_PROF_BACKPROJECT = 1
SP_PROF_PRECOND = 2
SP_PROF_TV = 3
SP_PROF_ITERATION = 4
SP_PROF_STORED_PROJECT = 5
SP_PROF_STORED_BACKPROJECT = 6

STATUS_NAMES = {
    SP_OK: "ok", SP_ERR_ARG: "invalid argument", SP_ERR_NOT_SPD: "preconditioner not SPD",
    SP_ERR_NONFINITE: "non-finite value", SP_ERR_HIP: "HIP error", SP_ERR_ALLOC: "allocation failed",
    SP_MAXITER: "max_iter reached", SP_CONVERGED: "converged",
    SP_BREAKDOWN_CONVERGED: "breakdown (exact step)", SP_TRIALS_EXHAUSTED: "trials exhausted",
}


class sp_geometry(ctypes.Structure):
    _fields_ = [("rows", c_int32), ("cols", c_int32), ("pixel", c_double),
                ("n_angles", c_int32), ("theta0", c_double), ("dtheta", c_double),
                ("n_bins", c_int32), ("bin_spacing", c_double), ("bin_offset", c_double)]


class sp_tv_params(ctypes.Structure):
    _fields_ = [("K", c_int32), ("a", c_double), ("gamma", c_double), ("max_trials", c_int32)]


class sp_precond(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("mu", c_double), ("rho", c_double), ("net", c_void_p)]


class sp_solve_params(ctypes.Structure):
    _fields_ = [("eps", c_double), ("max_iter", c_int32), ("flags", c_uint32),
                ("replay_trials", POINTER(c_int32))]


class sp_trace(ctypes.Structure):
    _fields_ = [("f_half", POINTER(c_double)), ("tv_half", POINTER(c_double)),
                ("alpha", POINTER(c_double)), ("beta", POINTER(c_double)),
                ("s_norm", POINTER(c_double)), ("ell", POINTER(c_int32)),
                ("trials", POINTER(c_int32)), ("cap", c_int32),
                ("f0", c_double), ("alpha0", c_double), ("fallbacks", c_int32),
                ("g_snap", c_void_p), ("g_snap_count", c_int32), ("bodies", c_int32),
                ("se_ref", c_void_p), ("se_axes", c_double * 2), ("se_c", c_double),
                ("se", POINTER(c_double)), ("se0", c_double), ("se1", c_double),
                ("t_ms", POINTER(c_double)), ("t1_ms", c_double)]


class sp_batch_trace(ctypes.Structure):
    _fields_ = [("f_half", POINTER(c_double)), ("tv_half", POINTER(c_double)),
                ("ell", POINTER(c_int32)), ("cap", c_int32), ("status", POINTER(c_int32))]


_SIGS = {
    "sp_version": (c_char_p, []),
    "sp_ctx_create": (c_int, [c_int, c_void_p, POINTER(c_void_p)]),
    "sp_ctx_destroy": (c_int, [c_void_p]),
    "sp_ctx_set_stream": (c_int, [c_void_p, c_void_p]),
    "sp_last_error": (c_char_p, [c_void_p]),
    "sp_ctx_last_error": (c_char_p, [c_void_p]),
    "sp_project": (c_int, [c_void_p, POINTER(sp_geometry), c_void_p, c_void_p]),
    "sp_backproject": (c_int, [c_void_p, POINTER(sp_geometry), c_void_p, c_void_p]),
    "sp_backproject_noalloc": (c_int, [c_void_p, POINTER(sp_geometry), c_void_p, c_void_p]),
    "sp_residual": (c_int, [c_void_p, POINTER(sp_geometry), c_void_p, c_void_p, c_void_p, c_void_p]),
    "sp_gradient": (c_int, [c_void_p, POINTER(sp_geometry), c_void_p, c_void_p, c_void_p, c_void_p]),
    "sp_precond_apply": (c_int, [c_void_p, POINTER(sp_geometry), POINTER(sp_precond), c_void_p, c_void_p]),
    "sp_tv": (c_int, [c_void_p, POINTER(sp_geometry), c_void_p, c_void_p]),
    "sp_selective_error": (c_int, [c_void_p, POINTER(sp_geometry), c_void_p, c_void_p,
                                   POINTER(c_double), c_double, c_void_p]),
    "sp_tv_grad": (c_int, [c_void_p, POINTER(sp_geometry), c_void_p, c_void_p, c_void_p]),
    "sp_tv_perturb": (c_int, [c_void_p, POINTER(sp_geometry), POINTER(sp_tv_params), c_void_p,
                              c_void_p, c_void_p, c_void_p, c_void_p]),
    "sp_suppcg_solve": (c_int, [c_void_p, POINTER(sp_geometry), c_void_p, c_void_p,
                                POINTER(sp_tv_params), POINTER(sp_precond), POINTER(sp_solve_params),
                                c_void_p, c_void_p, POINTER(c_int32), POINTER(sp_trace)]),
    "sp_suppcg_solve_batched": (c_int, [c_void_p, c_int32, POINTER(sp_geometry), POINTER(c_void_p),
                                        POINTER(c_void_p), POINTER(sp_tv_params), POINTER(sp_precond),
                                        POINTER(sp_solve_params), POINTER(c_void_p), POINTER(c_void_p),
                                        POINTER(c_int32), POINTER(sp_batch_trace)]),
    "sp_batch_tuning": (c_int, [c_void_p, POINTER(c_int32), c_int32]),
    "sp_state_save": (c_int, [c_void_p, c_void_p, POINTER(ctypes.c_int64)]),
    "sp_state_load": (c_int, [c_void_p, c_void_p, ctypes.c_int64]),
    "sp_solve_status": (c_int, [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32)]),
    "sp_lp_create": (c_int, [c_void_p, c_int32, c_int32, POINTER(c_void_p)]),
    "sp_lp_destroy": (c_int, [c_void_p]),
    "sp_lp_num_params": (ctypes.c_int64, [c_void_p]),
    "sp_lp_set_params": (c_int, [c_void_p, c_void_p, POINTER(ctypes.c_float), ctypes.c_int64]),
    "sp_lp_get_params": (c_int, [c_void_p, c_void_p, POINTER(ctypes.c_float), ctypes.c_int64]),
    "sp_lp_set_weights": (c_int, [c_void_p, c_void_p, POINTER(ctypes.c_float), ctypes.c_int64]),
    "sp_lp_get_weights": (c_int, [c_void_p, c_void_p, POINTER(ctypes.c_float), ctypes.c_int64]),
    "sp_lp_apply": (c_int, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p]),
    "sp_lp_loss_grad": (c_int, [c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_int32,
                                c_void_p, c_int32, c_int32, c_void_p, c_void_p]),
    "sp_lp_adam_step": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_double, c_double,
                                c_double, c_int32]),
    "sp_supart_solve": (c_int, [c_void_p, POINTER(sp_geometry), c_void_p, c_void_p, POINTER(sp_tv_params),
                                c_double, c_double, POINTER(sp_solve_params), c_void_p, POINTER(sp_trace)]),
    "sp_blobart_solve": (c_int, [c_void_p, POINTER(sp_geometry), c_void_p, c_double, c_double,
                                 POINTER(sp_solve_params), c_void_p, POINTER(sp_trace)]),
    "sp_tune_shapes": (c_int, [c_void_p, POINTER(sp_geometry), POINTER(c_int32), POINTER(c_int32),
                               POINTER(c_double)]),
    "sp_tuning_set": (c_int, [POINTER(sp_geometry), c_int32, c_int32]),
    "sp_tuning_list": (c_int, [POINTER(sp_geometry), POINTER(c_int32), POINTER(c_int32), c_int32,
                               POINTER(c_int32)]),
    "sp_tuning_clear": (c_int, []),
    "sp_matrix_build": (c_int, [c_void_p, POINTER(sp_geometry), POINTER(c_void_p)]),
    "sp_matrix_destroy": (c_int, [c_void_p]),
    "sp_matrix_info": (c_int, [c_void_p, POINTER(ctypes.c_int64), POINTER(ctypes.c_int64)]),
    "sp_matrix_project": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "sp_matrix_backproject": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "sp_matrix_export": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "sp_profile_enable": (c_int, [c_void_p, c_int]),
    "sp_profile_read": (c_int, [c_void_p, c_int, POINTER(c_double), POINTER(c_int32)]),
}

_lib = None


def load():
    """Loads libsuppcg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1807_10151_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGS)
