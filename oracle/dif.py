"""ctypes binding of the FP64 time-domain DIF oracle (``dif_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

The C source is compiled with the host ``gcc`` (``-O2``, no fast-math) into
``liboracle_dif.so`` next to it, on first use or when the source is newer.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dif_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_dif.so")

STOP_MAX_IMFS, STOP_FLOOR, STOP_FEW_EXTREMA = 0, 1, 2
FLAG_CAP = 1


class _Opts(ctypes.Structure):
    _fields_ = [
        ("mask_rule", ctypes.c_int32),
        ("inner_form", ctypes.c_int32),
        ("nu", ctypes.c_double),
        ("max_inner", ctypes.c_int64),
        ("floor_tau", ctypes.c_double),
    ]


class _Info(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int64),
        ("L", ctypes.c_int64),
        ("m", ctypes.c_int64),
        ("sd", ctypes.c_double),
        ("sd_prev", ctypes.c_double),
        ("margin_k", ctypes.c_double),
        ("floor_ratio", ctypes.c_double),
        ("flags", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc if needed; return the library path."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c99",
           "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        d = ctypes.POINTER(ctypes.c_double)
        lib.dif_count_extrema.restype = ctypes.c_int64
        lib.dif_count_extrema.argtypes = [d, ctypes.c_int64, d]
        lib.dif_mask_length.restype = ctypes.c_int64
        lib.dif_mask_length.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_double]
        lib.dif_window_column.restype = ctypes.c_int
        lib.dif_window_column.argtypes = [ctypes.c_int64, ctypes.c_int64, d]
        lib.dif_apply_window.restype = ctypes.c_int
        lib.dif_apply_window.argtypes = [d, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, d]
        lib.dif_inner_trace.restype = ctypes.c_int
        lib.dif_inner_trace.argtypes = [d, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.c_int64, d, d]
        lib.dif_decompose.restype = ctypes.c_int
        lib.dif_decompose.argtypes = [d, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                      ctypes.POINTER(_Opts), d, d,
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_Info),
                                      ctypes.POINTER(ctypes.c_int32)]
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def count_extrema(r) -> tuple[int, float]:
    """(k, margin): sign changes of the nonzero forward differences of r."""
    r = _f64(r)
    mg = np.zeros(1)
    k = _load().dif_count_extrema(_dp(r), r.size, _dp(mg))
    return int(k), float(mg[0])


def mask_length(N: int, k: int, rule: int = 0, nu: float = 1.6) -> int:
    return int(_load().dif_mask_length(N, k, rule, nu))


def window_column(N: int, L: int) -> np.ndarray:
    """First column of the circulant W: taps of (triangle * triangle)/L^4 folded mod N."""
    c = np.zeros(N)
    st = _load().dif_window_column(N, L, _dp(c))
    if st:
        raise RuntimeError("dif_window_column failed: %d" % st)
    return c


def apply_window(x, L: int, form: int = 0) -> np.ndarray:
    """W x (one periodic convolution with the window)."""
    x = _f64(x)
    a = np.zeros_like(x)
    st = _load().dif_apply_window(_dp(x), x.size, L, form, _dp(a))
    if st:
        raise RuntimeError("dif_apply_window failed: %d" % st)
    return a


def inner_trace(s, L: int, n_steps: int, form: int = 0):
    """Iterate (I - W) n_steps times; return (s_final, SD_1..SD_n, ||s_m - s_{m-1}||)."""
    x = _f64(s).copy()
    sd = np.zeros(max(n_steps, 1))
    st_norm = np.zeros(max(n_steps, 1))
    st = _load().dif_inner_trace(_dp(x), x.size, L, form, n_steps, _dp(sd), _dp(st_norm))
    if st:
        raise RuntimeError("dif_inner_trace failed: %d" % st)
    return x, sd[:n_steps], st_norm[:n_steps]


@dataclass
class Decomposition:
    imfs: np.ndarray                 # [n_imfs, N]
    remainder: np.ndarray            # [N]
    k: list = field(default_factory=list)
    L: list = field(default_factory=list)
    m: list = field(default_factory=list)
    sd: list = field(default_factory=list)
    sd_prev: list = field(default_factory=list)
    margin_k: list = field(default_factory=list)
    floor_ratio: list = field(default_factory=list)
    flags: list = field(default_factory=list)
    stop_reason: int = 0

    @property
    def n_imfs(self) -> int:
        return self.imfs.shape[0]


def decompose(s, delta: float, max_imfs: int, *, mask_rule: int = 0, nu: float = 1.6,
              max_inner: int = 1_000_000, floor_tau: float = 1e-9,
              inner_form: int | None = None) -> Decomposition:
    """Time-domain DIF decomposition of one signal (Algorithm 2), FP64.

    inner_form: 0 literal folded taps, 1 four periodic box sums; default picks
    the literal form for N <= 1024 and the box form above.
    """
    s = _f64(s)
    N = s.size
    if inner_form is None:
        inner_form = 0 if N <= 1024 else 1
    opts = _Opts(mask_rule, inner_form, nu, max_inner, floor_tau)
    imfs = np.zeros((max(max_imfs, 1), N))
    rem = np.zeros(N)
    n = ctypes.c_int32(0)
    reason = ctypes.c_int32(0)
    info = (_Info * max(max_imfs, 1))()
    st = _load().dif_decompose(_dp(s), N, delta, max_imfs, ctypes.byref(opts), _dp(imfs),
                               _dp(rem), ctypes.byref(n), info, ctypes.byref(reason))
    if st:
        raise RuntimeError("dif_decompose failed: %d" % st)
    nn = n.value
    out = Decomposition(imfs=imfs[:nn].copy(), remainder=rem, stop_reason=reason.value)
    for j in range(nn):
        out.k.append(int(info[j].k))
        out.L.append(int(info[j].L))
        out.m.append(int(info[j].m))
        out.sd.append(float(info[j].sd))
        out.sd_prev.append(float(info[j].sd_prev))
        out.margin_k.append(float(info[j].margin_k))
        out.floor_ratio.append(float(info[j].floor_ratio))
        out.flags.append(int(info[j].flags))
    return out
