"""Batched Fast Iterative Filtering (FIF) on MI355X (gfx950).

Python face of ``libfif.so`` (C ABI in ``include/fif.h``): it only
marshals torch device tensors and the current HIP stream into the library's
entry points; every step of the decomposition runs in hand-written HIP
kernels.  There is no CPU fallback: without a built library or a GPU the
calls raise.

    import torch, paper_1802_01359_amd as fif
    res = fif.decompose(x_cuda, delta=1e-3, max_imfs=8)          # one signal
    plan = fif.Plan(lengths, max_imfs=12)                         # a batch
    out = plan.run(packed_cuda, delta=1e-3)
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from ._binding import (EXPORTED, IMF_CAP, IMF_INFO_DTYPE, IMF_REFINED, FifError, Options, check, load,
                       LIB_PATH, STOP_FAILED, STOP_FEW_EXTREMA, STOP_FLOOR, STOP_MAX_IMFS)

__all__ = ["Options", "Plan", "BatchResult", "Decomposition", "decompose", "FifError", "IMF_CAP",
           "IMF_REFINED", "IMF_INFO_DTYPE", "EXPORTED", "LIB_PATH", "load"]


def _torch():
    import torch
    return torch


def _stream_ptr(torch) -> int:
    return int(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> int:
    return int(t.data_ptr()) if t is not None else 0


@dataclass
class Decomposition:
    imfs: "object"          # torch tensor [n_imfs, N] on the device
    remainder: "object"     # torch tensor [N]
    info: np.ndarray        # IMF_INFO_DTYPE [n_imfs]

    @property
    def n_imfs(self) -> int:
        return int(self.imfs.shape[0])


def decompose(signal, delta: float, max_imfs: int, options: Options | None = None,
              window: int = 0) -> Decomposition:
    """Plain single-signal form (fif_decompose / fif_decompose_f64).

    signal: 1-D contiguous torch tensor on the current GPU, float32 or float64.
    """
    torch = _torch()
    lib = load()
    if signal.dim() != 1 or not signal.is_cuda or not signal.is_contiguous():
        raise ValueError("signal must be a contiguous 1-D CUDA tensor")
    if signal.dtype not in (torch.float32, torch.float64):
        raise ValueError("signal must be float32 or float64")
    N = signal.numel()
    dev = signal.device
    imfs = torch.empty((max(max_imfs, 1), N), dtype=signal.dtype, device=dev)
    rem = torch.empty(N, dtype=signal.dtype, device=dev)
    n = torch.zeros(1, dtype=torch.int32, device=dev)
    info = torch.zeros(max(max_imfs, 1) * IMF_INFO_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    opt = (options or Options()).c()
    fn = lib.fif_decompose if signal.dtype == torch.float32 else lib.fif_decompose_f64
    with torch.cuda.device(dev):
        st = fn(_ptr(signal), N, window, float(delta), int(max_imfs), _ptr(imfs), _ptr(rem), _ptr(n),
                _ptr(info), ctypes.byref(opt), _stream_ptr(torch))
    check(st)
    k = int(n.item())
    inf = np.frombuffer(info.cpu().numpy().tobytes(), dtype=IMF_INFO_DTYPE)[:k].copy()
    return Decomposition(imfs=imfs[:k], remainder=rem, info=inf)


@dataclass
class BatchResult:
    imfs: "object"          # packed [max_imfs * sum N_b]
    remainders: "object"    # packed [sum N_b]
    n_imfs: "object"        # int32 [B] on the device
    sig_status: "object"    # int32 [B] on the device
    info_raw: "object"      # uint8 [B * max_imfs * 48] on the device
    lengths: np.ndarray
    offsets: np.ndarray
    max_imfs: int

    def info(self) -> np.ndarray:
        """IMF_INFO_DTYPE [B, max_imfs] (copied to the host)."""
        raw = self.info_raw.cpu().numpy().tobytes()
        return np.frombuffer(raw, dtype=IMF_INFO_DTYPE).reshape(len(self.lengths), self.max_imfs).copy()

    def imfs_of(self, b: int):
        """[max_imfs, N_b] view of signal b's IMF rows."""
        N = int(self.lengths[b])
        o = int(self.offsets[b]) * self.max_imfs
        return self.imfs[o:o + self.max_imfs * N].view(self.max_imfs, N)

    def remainder_of(self, b: int):
        o = int(self.offsets[b])
        return self.remainders[o:o + int(self.lengths[b])]


class Plan:
    """fif_plan_create / fif_decompose_batched for a fixed list of lengths."""

    def __init__(self, lengths, max_imfs: int, options: Options | None = None):
        torch = _torch()
        lib = load()
        self.lengths = np.asarray(lengths, dtype=np.int64).ravel()
        self.offsets = np.concatenate([[0], np.cumsum(self.lengths)]).astype(np.int64)
        self.max_imfs = int(max_imfs)
        self.total = int(self.offsets[-1])
        self._h = ctypes.c_void_p()
        arr = (ctypes.c_int64 * len(self.lengths))(*[int(v) for v in self.lengths])
        opt = (options or Options()).c()
        check(lib.fif_plan_create(ctypes.byref(self._h), arr, len(self.lengths), self.max_imfs,
                                  ctypes.byref(opt)))
        sz = ctypes.c_size_t()
        check(lib.fif_plan_workspace_size(self._h, ctypes.byref(sz)))
        self.workspace_bytes = int(sz.value)
        self.device = torch.cuda.current_device()
        self._ws = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                load().fif_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    def workspace(self):
        torch = _torch()
        if self._ws is None:
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device="cuda")
        return self._ws

    def alloc_outputs(self, dtype):
        torch = _torch()
        B = len(self.lengths)
        return BatchResult(
            imfs=torch.empty(self.max_imfs * self.total, dtype=dtype, device="cuda"),
            remainders=torch.empty(self.total, dtype=dtype, device="cuda"),
            n_imfs=torch.empty(B, dtype=torch.int32, device="cuda"),
            sig_status=torch.empty(B, dtype=torch.int32, device="cuda"),
            info_raw=torch.empty(B * self.max_imfs * IMF_INFO_DTYPE.itemsize, dtype=torch.uint8, device="cuda"),
            lengths=self.lengths, offsets=self.offsets, max_imfs=self.max_imfs)

    def profile(self, enable: bool = True) -> None:
        """Bracket every later kernel launch of this plan with HIP events."""
        check(load().fif_plan_profile(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        """{kind: (launches, total_ms)} accumulated since the last read (waits)."""
        from ._binding import KernelTime
        cap = 64
        arr = (KernelTime * cap)()
        n = ctypes.c_int32()
        check(load().fif_plan_profile_read(self._h, arr, cap, ctypes.byref(n)))
        return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(min(n.value, cap))}

    def run(self, signals, delta: float, out: BatchResult | None = None, with_info: bool = True) -> BatchResult:
        """Enqueue the batched decomposition on the current stream (async)."""
        torch = _torch()
        lib = load()
        if signals.dim() != 1 or signals.numel() != self.total or not signals.is_cuda \
                or not signals.is_contiguous():
            raise ValueError("signals must be a contiguous 1-D CUDA tensor of %d samples" % self.total)
        if out is None:
            out = self.alloc_outputs(signals.dtype)
        ws = self.workspace()
        base = _ptr(ws)
        aligned = (base + 255) // 256 * 256
        fn = lib.fif_decompose_batched if signals.dtype == torch.float32 else lib.fif_decompose_batched_f64
        check(fn(self._h, _ptr(signals), float(delta), _ptr(out.imfs), _ptr(out.remainders), _ptr(out.n_imfs),
                 _ptr(out.info_raw) if with_info else 0, _ptr(out.sig_status), aligned, _stream_ptr(torch)))
        return out


def release_cache() -> None:
    load().fif_release_cache()
