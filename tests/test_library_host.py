"""Host-side checks of libfif that need no GPU: the library loads, exports
every entry point include/fif.h declares, and rejects bad arguments on the
host before touching the device."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import siggen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fif.h")


def header_functions() -> set[str]:
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return set(re.findall(r"\b(fif_[a-z0-9_]+)\s*\(", text))


@pytest.fixture(scope="module")
def lib():
    from paper_1802_01359_amd import _binding
    if not os.path.exists(_binding.LIB_PATH):
        pytest.fail("libfif.so is not built; run __graft_entry__.build()")
    return _binding.load()


def test_exports_every_declared_symbol(lib):
    from paper_1802_01359_amd import _binding
    declared = header_functions()
    assert declared == set(_binding.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", _binding.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (fif_\w+)", out))
    assert declared <= exported, declared - exported
    for name in declared:
        assert hasattr(lib, name)


def test_options_default(lib):
    from paper_1802_01359_amd._binding import _Options
    o = _Options()
    lib.fif_options_default(ctypes.byref(o))
    assert (o.mask_rule, o.nu, o.max_inner, o.floor_tau) == (0, 1.6, 1_000_000, 1e-9)
    assert (o.stop_mode, o.gamma, o.peak_rho) == (0, 0.0, 0.1)
    assert (o.window, o.window_points) == (None, 0)
    assert o.precision == 0                                  # FIF_PREC_MIXED


def _plan_status(lib, lengths, max_imfs=4, **opt):
    from paper_1802_01359_amd._binding import Options
    h = ctypes.c_void_p()
    arr = (ctypes.c_int64 * max(len(lengths), 1))(*lengths)
    o = Options(**opt).c()
    return lib.fif_plan_create(ctypes.byref(h), arr, len(lengths), max_imfs, ctypes.byref(o))


@pytest.mark.parametrize("lengths,kw,status", [
    ([4096], dict(max_imfs=0), -1),
    ([4096], dict(max_imfs=5000), -1),
    ([1], {}, -1),
    ([0], {}, -1),
    ([4096, 11], {}, -2),            # prime factor 11
    ([4096, 8192 * 4096], {}, -2),    # 2^25 does not split into two factors <= 4096
    ([4099 * 2], {}, -2),              # 4099 is prime
    ([49 * 49 * 49 * 49 * 7], {}, -2),  # 7^9: no split into factors <= 8192
    ([4096], dict(mask_rule=3), -1),
    ([4096], dict(mask_rule=1, nu=-1.0), -1),
    ([4096], dict(max_inner=0), -1),
    ([4096], dict(floor_tau=-1.0), -1),
    ([4096], dict(stop_mode=3), -1),
    ([4096], dict(gamma=1.0), -1),
    ([4096], dict(gamma=-0.1), -1),
    ([4096], dict(mask_rule=2, peak_rho=0.0), -1),
    ([4096], dict(mask_rule=2, peak_rho=1.5), -1),
    ([4096], dict(window=[1.0]), -1),                 # fewer than two samples
    ([4096], dict(window=[0.0, 1.0]), -1),            # first sample not > 0
    ([4096], dict(window=[1.0, -0.5, 0.0]), -1),      # negative sample
    ([4096], dict(window=[1.0, float("nan")]), -1),
    ([4096], dict(window=np.ones(65538)), -1),        # too many samples
    ([4096], dict(window=[1.0, 0.0], stop_mode=2), -1),
    ([4096], dict(precision=2), -1),
    ([4096], dict(precision=1, window=[1.0, 0.0]), -1),   # the FP32 lane takes no window shape
    ([], {}, -1),
])
def test_plan_rejects_bad_arguments_on_host(lib, lengths, kw, status):
    max_imfs = kw.pop("max_imfs", 4)
    assert _plan_status(lib, lengths, max_imfs, **kw) == status
    assert lib.fif_last_error().decode() != ""


def test_single_rejects_bad_arguments_on_host(lib):
    from paper_1802_01359_amd._binding import Options
    o = Options().c()
    p = ctypes.c_void_p(1 << 20)  # never dereferenced: validation fails first
    # null buffers
    assert lib.fif_decompose(None, 64, 0, 1e-3, 4, p, p, p, None, ctypes.byref(o), None) == -1
    # bad window, delta, length, max_imfs
    assert lib.fif_decompose(p, 64, 7, 1e-3, 4, p, p, p, None, ctypes.byref(o), None) == -1
    assert lib.fif_decompose(p, 64, 0, 0.0, 4, p, p, p, None, ctypes.byref(o), None) == -1
    assert lib.fif_decompose(p, 64, 0, float("nan"), 4, p, p, p, None, ctypes.byref(o), None) == -1
    assert lib.fif_decompose(p, 1, 0, 1e-3, 4, p, p, p, None, ctypes.byref(o), None) == -1
    assert lib.fif_decompose(p, 13, 0, 1e-3, 4, p, p, p, None, ctypes.byref(o), None) == -2
    assert lib.fif_decompose(p, 64, 0, 1e-3, 0, p, p, p, None, ctypes.byref(o), None) == -1
    bad = Options(max_inner=0).c()
    assert lib.fif_decompose(p, 64, 0, 1e-3, 4, p, p, p, None, ctypes.byref(bad), None) == -1
    # the window argument and the options' samples must agree
    assert lib.fif_decompose(p, 64, 1, 1e-3, 4, p, p, p, None, ctypes.byref(o), None) == -1
    w = Options(window=[1.0, 0.5, 0.0]).c()
    assert lib.fif_decompose(p, 64, 0, 1e-3, 4, p, p, p, None, ctypes.byref(w), None) == -1


def test_batched_rejects_null_plan(lib):
    p = ctypes.c_void_p(1 << 20)
    assert lib.fif_decompose_batched(None, p, 1e-3, p, p, p, None, None, p, None) == -1


def test_uneven_lengths_are_smooth():
    L = siggen.uneven_lengths(512)
    assert L.min() >= 1024 and L.max() <= 262144
    for n in L[:64]:
        n = int(n)
        for q in (2, 3, 5, 7):
            while n % q == 0:
                n //= q
        assert n == 1
    # log-uniform: roughly half the lengths below the geometric midpoint 16384
    assert 0.35 < np.mean(L < 16384) < 0.65
