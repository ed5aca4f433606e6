"""ctypes binding of the C ABI in ``include/sft.h`` (argument marshalling only).

Every function here has the name of the C entry point it calls and forwards
its arguments unchanged; all computation happens in ``libsft.so``.  Loading
fails loudly if the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsft.so")

SFT_OK = 0
SFT_ERR_ARG, SFT_ERR_SHAPE, SFT_ERR_OOM, SFT_ERR_HIP = -1, -2, -3, -4
SFT_ERR_NOT_FINITE, SFT_ERR_STATE, SFT_ERR_UNSUPPORTED = -5, -6, -7
SFT_FP64, SFT_FP32_MIXED = 0, 1
SFT_WENO3CSH, SFT_UPWIND = 0, 1
SFT_SSPRK43, SFT_FE, SFT_SSPRK33 = 0, 1, 2
SFT_RKG2, SFT_RKL2, SFT_DIFF_FE = 0, 1, 2
SFT_DTYPE_F64, SFT_DTYPE_F32 = 0, 1
SFT_WEIGHT_F, SFT_WEIGHT_MU, SFT_WEIGHT_DISK = 0, 1, 2
SFT_KFAM_STS_STAGE, SFT_KFAM_STS_FIRST, SFT_KFAM_ADV_STAGE = 0, 1, 2
SFT_KFAM_ASSIM, SFT_KFAM_DIAG, SFT_KFAM_OTHER, SFT_KFAM_SOURCE, SFT_KFAM_COUNT = 3, 4, 5, 6, 7
KFAM_NAMES = ("sts_stage", "sts_first", "adv_stage", "assim", "diag", "other", "source")


class sft_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("adv_scheme", ctypes.c_int32),
                ("adv_time", ctypes.c_int32), ("diff_time", ctypes.c_int32),
                ("cfl_safety", ctypes.c_double), ("dt_max", ctypes.c_double),
                ("ptl_dt", ctypes.c_double), ("use_graphs", ctypes.c_int32),
                ("sts_fuse", ctypes.c_int32), ("diag_every_call", ctypes.c_int32),
                ("sts_tile", ctypes.c_int32), ("strang", ctypes.c_int32),
                ("rfe_model", ctypes.c_int32), ("rfe_seed", ctypes.c_uint32), ("lanes", ctypes.c_int32),
                ("rfe_phi_hr", ctypes.c_double), ("rfe_lifetime_h", ctypes.c_double),
                ("dt_min", ctypes.c_double), ("att_cfl", ctypes.c_int32), ("reserved0", ctypes.c_int32)]


class sft_params(ctypes.Structure):
    _fields_ = [("nu_km2_s", ctypes.c_double), ("d0", ctypes.c_double), ("d2", ctypes.c_double),
                ("d4", ctypes.c_double), ("m1", ctypes.c_double), ("m3", ctypes.c_double),
                ("m5", ctypes.c_double), ("alpha_mu", ctypes.c_double), ("mu_lim", ctypes.c_double),
                ("lat_lim_deg", ctypes.c_double), ("flux_balance", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("att_b0", ctypes.c_double),
                ("nu_grid_alpha", ctypes.c_double)]


class sft_diag(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt_last", ctypes.c_double), ("steps", ctypes.c_int64),
                ("stages", ctypes.c_int64), ("phi_pos", ctypes.c_double),
                ("phi_neg", ctypes.c_double), ("phi_net", ctypes.c_double), ("h1", ctypes.c_double),
                ("h2", ctypes.c_double), ("dax", ctypes.c_double), ("bmin", ctypes.c_double),
                ("bmax", ctypes.c_double), ("babs_min", ctypes.c_double),
                ("nonfinite", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("surr_accept", ctypes.c_int64), ("surr_reject", ctypes.c_int64)]


_P = ctypes.c_void_p
_I = ctypes.c_int32
_D = ctypes.c_double
_PI = ctypes.POINTER(ctypes.c_int32)
_PI64 = ctypes.POINTER(ctypes.c_int64)

# name -> (restype, argtypes); every symbol declared in include/sft.h
SIGNATURES = {
    "sft_options_default": (_I, [ctypes.POINTER(sft_options)]),
    "sft_create": (_I, [ctypes.POINTER(_P), ctypes.POINTER(sft_options), _P]),
    "sft_add_grid": (_I, [_P, _I, _I, _PI]),
    "sft_add_realizations": (_I, [_P, _I, _I, ctypes.POINTER(sft_params), _PI]),
    "sft_set_state": (_I, [_P, _I, _P, _I, _I]),
    "sft_get_state": (_I, [_P, _I, _P, _I, _I]),
    "sft_set_states": (_I, [_P, _I, _P, _I, _I]),
    "sft_get_states": (_I, [_P, _I, _P, _I, _I]),
    "sft_advance": (_I, [_P, _D]),
    "sft_assimilate": (_I, [_P, _I, _P, _P, _I, _I, _D, _D, _I]),
    "sft_assimilate_noalloc": (_I, [_P, _I, _P, _P, _I, _I, _D, _D]),
    "sft_diagnostics": (_I, [_P, _I, ctypes.POINTER(sft_diag)]),
    "sft_time": (_I, [_P, ctypes.POINTER(_D)]),
    "sft_set_time": (_I, [_P, _D]),
    "sft_sync": (_I, [_P]),
    "sft_counts": (_I, [_P, _I, _PI64, _PI64, _PI64, _PI64]),
    "sft_set_timing": (_I, [_P, _I]),
    "sft_get_timing": (_I, [_P, _I, ctypes.POINTER(_D), _PI64, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "sft_tile_info": (_I, [_I, _I, _PI, _PI, _PI, _PI]),
    "sft_tile_choice": (_I, [_P, _I, _PI]),
    "sft_set_class_tile": (_I, [_P, _I, _I]),
    "sft_destroy": (_I, [_P]),
    "sft_net_create": (_I, [ctypes.POINTER(_P), _I, _I, _I, _P]),
    "sft_net_param_count": (_I, [_P, _PI64]),
    "sft_net_set_params": (_I, [_P, _P, _I]),
    "sft_net_get_params": (_I, [_P, _P, _I]),
    "sft_net_get_grads": (_I, [_P, _P, _I]),
    "sft_net_forward": (_I, [_P, _I, _P, _I, _P, _P]),
    "sft_net_predict": (_I, [_P, _I, _P, _I, _P, _P]),
    "sft_net_get_activation": (_I, [_P, _I, _P]),
    "sft_net_train_step": (_I, [_P, _I, _P, _P, _I, _P, ctypes.c_float, _I, ctypes.POINTER(_D)]),
    "sft_net_set_grid_limit": (_I, [_P, _I]),
    "sft_net_sync": (_I, [_P]),
    "sft_net_destroy": (_I, [_P]),
    "sft_surrogate_advance": (_I, [_P, _I, _P, _P, _D, _D, _I, ctypes.POINTER(_D)]),
    "sft_surrogate_counts": (_I, [_P, _I, _PI64, _PI64, _PI64, _PI]),
    "sft_status_string": (ctypes.c_char_p, [_I]),
    "sft_last_error": (ctypes.c_char_p, [_P]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libsft.so (raises if it is missing: build it with build.py)."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: torch ships its own libamdhip64 and
        # HSA runtime.  Loaded first, they satisfy this library's
        # libamdhip64.so.7 dependency by soname, so device pointers and
        # streams of torch tensors are valid here; loaded after this library,
        # a second runtime would claim the device and torch could not use it.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library {LIB_PATH} is missing; build it with "
                "`python -m paper_2501_06377_amd.build` (hipcc, gfx950). No CPU fallback exists.")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class SftError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def check(status: int, ctx=None, what: str = "") -> int:
    if status != SFT_OK:
        L = load()
        text = L.sft_status_string(status).decode()
        detail = L.sft_last_error(ctx).decode() if ctx else ""
        raise SftError(status, f"{what}: {text}" + (f": {detail}" if detail else ""))
    return status
