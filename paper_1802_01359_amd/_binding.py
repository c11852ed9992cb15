"""ctypes binding of libfif (argument marshalling only).

Every step of the decomposition runs in the library's HIP kernels; torch is
used for device memory and the current HIP stream.  Loading fails loudly
when libfif.so has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfif.so")

FIF_OK = 0
FIF_ERR_INVALID_ARG = -1
FIF_ERR_UNSUPPORTED_LENGTH = -2
FIF_ERR_NOMEM = -3
FIF_ERR_DEVICE = -4
FIF_ERR_NONFINITE = -5
FIF_ERR_CAPACITY = -6
FIF_ERR_NOT_FOUND = -7

# size of the library's static workspace (fif_decompose_batched_static)
STATIC_WORKSPACE_BYTES = 64 << 20

IMF_CAP = 1
IMF_REFINED = 2

# fif_options.precision
PREC_MIXED, PREC_FP32 = 0, 1

STOP_MAX_IMFS, STOP_FLOOR, STOP_FEW_EXTREMA, STOP_FAILED = 0, 1, 2, 3

# symbols declared in include/fif.h
EXPORTED = (
    "fif_options_default", "fif_last_error", "fif_status_string",
    "fif_plan_create", "fif_plan_workspace_size", "fif_plan_destroy",
    "fif_decompose_batched", "fif_decompose_batched_f64",
    "fif_decompose", "fif_decompose_f64", "fif_release_cache",
    "fif_plan_profile", "fif_plan_profile_read",
    "fif_model_create", "fif_model_free", "fif_model_get_params", "fif_model_set_params",
    "fif_model_save", "fif_model_load", "fif_model_forward", "fif_model_grad", "fif_model_train_step",
    "fif_plan_set_proposal", "fif_plan_record_features", "fif_decompose_batched_graph",
    "fif_decompose_batched_graph_f64", "fif_decompose_batched_static",
    "fif_plan_create_tuned", "fif_plan_length_plan", "fif_tune_cache_lookup", "fif_tune_cache_store",
    "fif_device_tune_key",
)

NET_FEATURES = 1024
NET_CHANNELS = 8
NET_PARAMS = 147458


class FifError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("fif status %d: %s" % (status, message))
        self.status = status


class _Options(ctypes.Structure):
    _fields_ = [("mask_rule", ctypes.c_int32), ("stop_mode", ctypes.c_int32), ("nu", ctypes.c_double),
                ("max_inner", ctypes.c_int64), ("floor_tau", ctypes.c_double), ("gamma", ctypes.c_double),
                ("peak_rho", ctypes.c_double), ("window", ctypes.c_void_p), ("window_points", ctypes.c_int32),
                ("precision", ctypes.c_int32)]


class LengthPlan(ctypes.Structure):
    """fif_length_plan: how one signal length is transformed."""
    _fields_ = [("N", ctypes.c_int64), ("N1", ctypes.c_int32), ("N2", ctypes.c_int32), ("TC", ctypes.c_int32),
                ("TR", ctypes.c_int32), ("n_rad1", ctypes.c_int32), ("n_rad2", ctypes.c_int32),
                ("rad1", ctypes.c_int8 * 24), ("rad2", ctypes.c_int8 * 24), ("us", ctypes.c_double),
                ("us_default", ctypes.c_double)]

    def to_dict(self) -> dict:
        return {"N": int(self.N), "N1": int(self.N1), "N2": int(self.N2), "TC": int(self.TC), "TR": int(self.TR),
                "rad1": [int(self.rad1[i]) for i in range(self.n_rad1)],
                "rad2": [int(self.rad2[i]) for i in range(self.n_rad2)], "us": float(self.us),
                "us_default": float(self.us_default)}

    @classmethod
    def from_dict(cls, d: dict) -> "LengthPlan":
        c = cls()
        c.N, c.N1, c.N2, c.TC, c.TR = int(d["N"]), int(d["N1"]), int(d["N2"]), int(d["TC"]), int(d["TR"])
        r1, r2 = list(d.get("rad1", [])), list(d.get("rad2", []))
        c.n_rad1, c.n_rad2 = len(r1), len(r2)
        for i, r in enumerate(r1[:24]):
            c.rad1[i] = int(r)
        for i, r in enumerate(r2[:24]):
            c.rad2[i] = int(r)
        c.us, c.us_default = float(d.get("us", 0.0)), float(d.get("us_default", 0.0))
        return c


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


IMF_INFO_DTYPE = np.dtype([("k", "<i8"), ("L", "<i8"), ("m", "<i8"), ("sd", "<f8"), ("sd_prev", "<f8"),
                           ("flags", "<u4"), ("evals", "<u4")])
assert IMF_INFO_DTYPE.itemsize == 48


@dataclass
class Options:
    mask_rule: int = 0          # 0 ceil(2N/k), 1 2*floor(nu*N/k), 2 spectral peak
    nu: float = 1.6
    max_inner: int = 1_000_000
    floor_tau: float = 1e-9
    stop_mode: int = 0          # 0 SD <= delta, 1 ||s_{m+1}-s_m|| < delta, 2 a-priori N0
    gamma: float = 0.0          # > 0: thresholded IMF
    peak_rho: float = 0.1
    window: object = None       # samples of a window shape on [0, 1]; None: the triangle
    precision: int = 0          # PREC_MIXED (FP64 transforms) or PREC_FP32 (the FP32 lane, no parity claim)

    def c(self) -> _Options:
        o = _Options(self.mask_rule, self.stop_mode, self.nu, self.max_inner, self.floor_tau, self.gamma,
                     self.peak_rho, None, 0, self.precision)
        if self.window is not None:
            w = np.ascontiguousarray(np.asarray(self.window, dtype=np.float64).ravel())
            o.window = w.ctypes.data
            o.window_points = w.size
            o._keep = w             # the library copies the samples during the call
        return o


_lib = None


def load():
    """Load libfif.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libfif.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.fif_options_default.argtypes = [ctypes.POINTER(_Options)]
    lib.fif_options_default.restype = None
    lib.fif_last_error.restype = ctypes.c_char_p
    lib.fif_last_error.argtypes = []
    lib.fif_status_string.restype = ctypes.c_char_p
    lib.fif_status_string.argtypes = [ctypes.c_int]
    lib.fif_plan_create.restype = ctypes.c_int
    lib.fif_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(i64), i32, i32, ctypes.POINTER(_Options)]
    lib.fif_plan_create_tuned.restype = ctypes.c_int
    lib.fif_plan_create_tuned.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(i64), i32, i32, ctypes.POINTER(_Options),
                                          ctypes.c_char_p]
    lib.fif_plan_length_plan.restype = ctypes.c_int
    lib.fif_plan_length_plan.argtypes = [vp, i64, ctypes.POINTER(LengthPlan)]
    lib.fif_tune_cache_lookup.restype = ctypes.c_int
    lib.fif_tune_cache_lookup.argtypes = [ctypes.c_char_p, ctypes.c_char_p, i64, ctypes.POINTER(LengthPlan)]
    lib.fif_tune_cache_store.restype = ctypes.c_int
    lib.fif_tune_cache_store.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(LengthPlan)]
    lib.fif_device_tune_key.restype = ctypes.c_int
    lib.fif_device_tune_key.argtypes = [ctypes.c_char_p, i32]
    lib.fif_plan_workspace_size.restype = ctypes.c_int
    lib.fif_plan_workspace_size.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.fif_plan_destroy.restype = ctypes.c_int
    lib.fif_plan_destroy.argtypes = [vp]
    for name in ("fif_decompose_batched", "fif_decompose_batched_f64", "fif_decompose_batched_graph",
                 "fif_decompose_batched_graph_f64"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [vp, vp, dbl, vp, vp, vp, vp, vp, vp, vp]
    lib.fif_decompose_batched_static.restype = ctypes.c_int
    lib.fif_decompose_batched_static.argtypes = [vp, vp, dbl, vp, vp, vp, vp, vp, vp]
    for name in ("fif_decompose", "fif_decompose_f64"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [vp, i64, ctypes.c_int, dbl, i32, vp, vp, vp, vp, ctypes.POINTER(_Options), vp]
    lib.fif_release_cache.restype = None
    lib.fif_release_cache.argtypes = []
    lib.fif_plan_profile.restype = ctypes.c_int
    lib.fif_plan_profile.argtypes = [vp, i32]
    lib.fif_plan_profile_read.restype = ctypes.c_int
    lib.fif_plan_profile_read.argtypes = [vp, ctypes.POINTER(KernelTime), i32, ctypes.POINTER(i32)]
    fp = ctypes.POINTER(ctypes.c_float)
    lib.fif_model_create.restype = ctypes.c_int
    lib.fif_model_create.argtypes = [ctypes.POINTER(vp), fp, i32]
    lib.fif_model_free.restype = ctypes.c_int
    lib.fif_model_free.argtypes = [vp]
    lib.fif_model_get_params.restype = ctypes.c_int
    lib.fif_model_get_params.argtypes = [vp, fp]
    lib.fif_model_set_params.restype = ctypes.c_int
    lib.fif_model_set_params.argtypes = [vp, fp]
    lib.fif_model_save.restype = ctypes.c_int
    lib.fif_model_save.argtypes = [vp, ctypes.c_char_p]
    lib.fif_model_load.restype = ctypes.c_int
    lib.fif_model_load.argtypes = [ctypes.POINTER(vp), ctypes.c_char_p, i32]
    lib.fif_model_forward.restype = ctypes.c_int
    lib.fif_model_forward.argtypes = [vp, vp, i32, vp, vp]
    lib.fif_model_grad.restype = ctypes.c_int
    lib.fif_model_grad.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    lib.fif_model_train_step.restype = ctypes.c_int
    lib.fif_model_train_step.argtypes = [vp, vp, vp, i32, ctypes.c_float, vp, vp]
    lib.fif_plan_set_proposal.restype = ctypes.c_int
    lib.fif_plan_set_proposal.argtypes = [vp, vp]
    lib.fif_plan_record_features.restype = ctypes.c_int
    lib.fif_plan_record_features.argtypes = [vp, vp]
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != FIF_OK:
        msg = load().fif_last_error().decode(errors="replace")
        raise FifError(status, msg)
