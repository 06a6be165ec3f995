"""ctypes binding of libopentm_amd.so (the C ABI in include/opentm_amd.h).

Argument marshalling only: every step of the homogenization path runs in the
library's HIP kernels.  There is no CPU fallback; loading fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(PKG, "libopentm_amd.so")

OTM_OK = 0
OTM_NOT_CONVERGED = 1
OTM_EINVAL = -1
OTM_ENOMEM = -2
OTM_EDEVICE = -3
OTM_ENONFINITE = -4
OTM_EUNSUPPORTED = -5
OTM_ESTATE = -6
OTM_EIO = -7

OTM_FP64 = 0
OTM_MIXED = 1
OTM_GUESS_ZERO = 0
OTM_GUESS_PREVIOUS = 1
OTM_GUESS_USER = 2
OTM_GUESS_LEARNED = 3
OTM_PRECOND_JACOBI = 0
OTM_PRECOND_MG = 1
OTM_MG_JACOBI = 0
OTM_MG_GS8 = 1
OTM_OBJ_MSE = 0
OTM_OBJ_REL = 1
OTM_OBJ_L1 = 2
OTM_INIT_P = 0
OTM_INIT_D = 1
OTM_INIT_G = 2
OTM_INIT_IWP = 3
OTM_INIT_BALL = 4
OTM_SYM_NONE = 0
OTM_SYM_CENTRAL = 1

FIELDS = {"rho": 0, "rhof": 1, "k": 2, "b": 3, "diag": 4, "chi": 5, "sens_elem": 6, "sens": 7}
FIELD3 = {"b", "chi"}

# Every symbol include/opentm_amd.h declares.
EXPORTED = [
    "otm_default_options", "otm_create", "otm_destroy", "otm_set_density", "otm_set_density_device",
    "otm_homogenize", "otm_sensitivity", "otm_oc_update", "otm_step", "otm_optimize", "otm_get_field",
    "otm_set_field", "otm_set_guess", "otm_get_governor", "otm_set_governor", "otm_apply", "otm_prepare", "otm_apply_device",
    "otm_time_apply_device", "otm_get_tile", "otm_pass_timing", "otm_get_timings", "otm_strerror", "otm_last_error", "otm_version",
    "otm_batch_create", "otm_batch_destroy", "otm_batch_set_density", "otm_batch_get_field", "otm_batch_step",
    "otm_batch_set_graph", "otm_batch_info", "otm_batch_last_error",
    "otm_nn_create", "otm_nn_destroy", "otm_nn_param_count", "otm_nn_get_params", "otm_nn_set_params",
    "otm_nn_get_grads", "otm_nn_forward", "otm_nn_accumulate", "otm_nn_adam", "otm_nn_zero_grads",
    "otm_nn_last_error", "otm_set_network", "otm_init_density", "otm_apply_device_tiled", "otm_device_bytes",
    "otm_batch_device_bytes", "otm_batch_get_governor", "otm_oc_update_noalloc",
    "otm_save_state", "otm_load_state", "otm_nn_save", "otm_nn_load", "otm_batch_save_state",
    "otm_batch_load_state",
]


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("k0", ctypes.c_double), ("kmin", ctypes.c_double),
                ("penal", ctypes.c_double), ("filter_radius", ctypes.c_double),
                ("target", ctypes.c_double * 6), ("vf", ctypes.c_double), ("objective", ctypes.c_int32),
                ("symmetry", ctypes.c_int32)]


class SolverOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("guess", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32), ("reliable_delta", ctypes.c_double),
                ("kernel_variant", ctypes.c_int32), ("tile_tz", ctypes.c_int32), ("tile_tx", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("preconditioner", ctypes.c_int32), ("mg_sweeps", ctypes.c_int32),
                ("mg_coarse_sweeps", ctypes.c_int32), ("stall_window", ctypes.c_int32),
                ("mg_smoother", ctypes.c_int32)]


class OcOpts(ctypes.Structure):
    _fields_ = [("move", ctypes.c_double), ("eta", ctypes.c_double), ("rho_min", ctypes.c_double),
                ("move_min", ctypes.c_double)]


class GovernorOpts(ctypes.Structure):
    _fields_ = [("bound", ctypes.c_double), ("dg_small", ctypes.c_double), ("dv_small", ctypes.c_double),
                ("decay", ctypes.c_double), ("rebound", ctypes.c_double), ("g_tol", ctypes.c_double),
                ("patience", ctypes.c_int32), ("stall_iters", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32 * 3), ("rel_residual", ctypes.c_double * 3),
                ("converged", ctypes.c_int32), ("refreshes", ctypes.c_int32), ("ms_solve", ctypes.c_double),
                ("stalled", ctypes.c_int32), ("fallback", ctypes.c_int32)]


class IterRecord(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int32), ("g", ctypes.c_double), ("kappa", ctypes.c_double * 6),
                ("volume", ctypes.c_double), ("low_bound", ctypes.c_double), ("vstar", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("pcg_iters", ctypes.c_int32 * 3),
                ("rel_residual", ctypes.c_double * 3), ("ms_total", ctypes.c_double),
                ("ms_solve", ctypes.c_double), ("stop", ctypes.c_int32), ("move", ctypes.c_double),
                ("stalled", ctypes.c_int32)]

    def to_dict(self):
        return dict(iter=self.iter, g=self.g, kappa=list(self.kappa), volume=self.volume,
                    low_bound=self.low_bound, vstar=self.vstar, lam=self.lambda_,
                    pcg_iters=list(self.pcg_iters), rel_residual=list(self.rel_residual),
                    ms_total=self.ms_total, ms_solve=self.ms_solve, stop=self.stop, move=self.move,
                    stalled=self.stalled)


_lib = None


class OTMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"opentm status {status}: {msg}")
        self.status = status


def lib():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError(f"HIP library not built: {LIBPATH} is missing "
                           "(run `python -c 'import __graft_entry__ as g; g.build()'`)")
    L = ctypes.CDLL(LIBPATH)
    P = ctypes.POINTER
    dp = P(ctypes.c_double)
    vp = ctypes.c_void_p
    ctx = vp
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    sig = {
        "otm_default_options": ([P(SolverOpts), P(OcOpts), P(GovernorOpts)], None),
        "otm_create": ([P(Problem), P(SolverOpts), P(OcOpts), P(GovernorOpts), vp, P(vp)], ctypes.c_int),
        "otm_destroy": ([ctx], None),
        "otm_set_density": ([ctx, dp, i64], ctypes.c_int),
        "otm_set_density_device": ([ctx, vp, i64], ctypes.c_int),
        "otm_homogenize": ([ctx, dp, P(SolveStats)], ctypes.c_int),
        "otm_sensitivity": ([ctx, dp, dp], ctypes.c_int),
        "otm_oc_update": ([ctx, ctypes.c_double, dp, dp], ctypes.c_int),
        "otm_oc_update_noalloc": ([i32, vp, vp, ctypes.c_double, P(OcOpts), vp, vp, vp], ctypes.c_int),
        "otm_step": ([ctx, P(IterRecord)], ctypes.c_int),
        "otm_optimize": ([ctx, i32, dp, P(IterRecord), i32, P(i32)], ctypes.c_int),
        "otm_get_field": ([ctx, i32, dp, i64], ctypes.c_int),
        "otm_set_field": ([ctx, i32, dp, i64], ctypes.c_int),
        "otm_set_guess": ([ctx, dp, i64], ctypes.c_int),
        "otm_get_governor": ([ctx, dp], ctypes.c_int),
        "otm_set_governor": ([ctx, dp], ctypes.c_int),
        "otm_apply": ([ctx, i32, dp, dp], ctypes.c_int),
        "otm_prepare": ([ctx], ctypes.c_int),
        "otm_apply_device": ([i32, i32, i32, vp, vp, vp, vp], ctypes.c_int),
        "otm_apply_device_tiled": ([i32, i32, i32, i32, i32, vp, vp, vp, vp], ctypes.c_int),
        "otm_time_apply_device": ([i32, i32, i32, i32, i32, vp, vp, vp, vp, i32, dp], ctypes.c_int),
        "otm_get_timings": ([ctx, dp], ctypes.c_int),
        "otm_device_bytes": ([ctx, P(ctypes.c_int64)], ctypes.c_int),
        "otm_batch_device_bytes": ([vp, P(ctypes.c_int64)], ctypes.c_int),
        "otm_get_tile": ([ctx, P(i32)], ctypes.c_int),
        "otm_pass_timing": ([ctx, i32, dp], ctypes.c_int),
        "otm_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "otm_last_error": ([ctx], ctypes.c_char_p),
        "otm_version": ([], ctypes.c_char_p),
        "otm_init_density": ([i32, i32, ctypes.c_double, dp], ctypes.c_int),
        "otm_batch_create": ([P(Problem), i32, P(SolverOpts), P(OcOpts), P(GovernorOpts), vp, P(vp)], ctypes.c_int),
        "otm_batch_destroy": ([vp], None),
        "otm_batch_set_density": ([vp, i32, dp, i64], ctypes.c_int),
        "otm_batch_get_field": ([vp, i32, i32, dp, i64], ctypes.c_int),
        "otm_batch_step": ([vp, P(IterRecord)], ctypes.c_int),
        "otm_batch_set_graph": ([vp, i32], ctypes.c_int),
        "otm_batch_info": ([vp, dp], ctypes.c_int),
        "otm_batch_get_governor": ([vp, i32, dp], ctypes.c_int),
        "otm_batch_last_error": ([vp], ctypes.c_char_p),
        "otm_nn_create": ([i32, ctypes.c_uint64, vp, P(vp)], ctypes.c_int),
        "otm_nn_destroy": ([vp], None),
        "otm_nn_param_count": ([], i32),
        "otm_nn_get_params": ([vp, P(ctypes.c_float), i64], ctypes.c_int),
        "otm_nn_set_params": ([vp, P(ctypes.c_float), i64], ctypes.c_int),
        "otm_nn_get_grads": ([vp, P(ctypes.c_float), i64], ctypes.c_int),
        "otm_nn_forward": ([vp, i32, vp, vp], ctypes.c_int),
        "otm_nn_accumulate": ([vp, i32, vp, vp, dp], ctypes.c_int),
        "otm_nn_adam": ([vp, ctypes.c_double, i32], ctypes.c_int),
        "otm_nn_zero_grads": ([vp], ctypes.c_int),
        "otm_nn_last_error": ([vp], ctypes.c_char_p),
        "otm_set_network": ([vp, vp], ctypes.c_int),
        "otm_save_state": ([ctx, ctypes.c_char_p], ctypes.c_int),
        "otm_batch_save_state": ([vp, ctypes.c_char_p], ctypes.c_int),
        "otm_batch_load_state": ([vp, ctypes.c_char_p], ctypes.c_int),
        "otm_load_state": ([ctx, ctypes.c_char_p], ctypes.c_int),
        "otm_nn_save": ([vp, ctypes.c_char_p], ctypes.c_int),
        "otm_nn_load": ([vp, ctypes.c_char_p], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(status: int, ctx=None, allow_not_converged: bool = True) -> int:
    if status == OTM_OK or (status == OTM_NOT_CONVERGED and allow_not_converged):
        return status
    L = lib()
    msg = L.otm_strerror(status).decode()
    if ctx is not None:
        detail = L.otm_last_error(ctx).decode()
        if detail:
            msg += f" ({detail})"
    raise OTMError(status, msg)


def default_options():
    s, o, g = SolverOpts(), OcOpts(), GovernorOpts()
    lib().otm_default_options(ctypes.byref(s), ctypes.byref(o), ctypes.byref(g))
    return s, o, g
