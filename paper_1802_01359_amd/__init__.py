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

from ._binding import (EXPORTED, IMF_CAP, PREC_FP32, PREC_MIXED, STATIC_WORKSPACE_BYTES, LengthPlan, IMF_INFO_DTYPE, IMF_REFINED, NET_CHANNELS, NET_FEATURES, NET_PARAMS,
                       FifError, Options, check, load, LIB_PATH, STOP_FAILED, STOP_FEW_EXTREMA, STOP_FLOOR,
                       STOP_MAX_IMFS)

__all__ = ["Options", "Plan", "BatchResult", "Decomposition", "decompose", "FifError", "IMF_CAP",
           "IMF_REFINED", "IMF_INFO_DTYPE", "EXPORTED", "LIB_PATH", "load", "Model", "NET_PARAMS",
           "NET_FEATURES", "NET_CHANNELS", "PREC_MIXED", "PREC_FP32"]


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
              window: int | None = None) -> Decomposition:
    """Plain single-signal form (fif_decompose / fif_decompose_f64).

    signal: 1-D contiguous torch tensor on the current GPU, float32 or float64.
    window: fif_window value; by default FIF_WINDOW_SAMPLED when the options
    carry window samples, else FIF_WINDOW_TRI2.
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
    options = options or Options()
    if window is None:
        window = 1 if options.window is not None else 0
    opt = options.c()
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

    def __init__(self, lengths, max_imfs: int, options: Options | None = None, tune: bool = False,
                 tune_cache: str | None = None):
        """tune / tune_cache: fif_plan_create_tuned (measured choices of split,
        tiles and radix order per length, cached in the file tune_cache)."""
        torch = _torch()
        lib = load()
        self.lengths = np.asarray(lengths, dtype=np.int64).ravel()
        self.offsets = np.concatenate([[0], np.cumsum(self.lengths)]).astype(np.int64)
        self.max_imfs = int(max_imfs)
        self.B = len(self.lengths)
        self.total = int(self.offsets[-1])
        self._h = ctypes.c_void_p()
        arr = (ctypes.c_int64 * len(self.lengths))(*[int(v) for v in self.lengths])
        opt = (options or Options()).c()
        if tune or tune_cache is not None:
            check(lib.fif_plan_create_tuned(ctypes.byref(self._h), arr, len(self.lengths), self.max_imfs,
                                            ctypes.byref(opt), tune_cache.encode() if tune_cache else None))
        else:
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

    def length_plan(self, N: int) -> dict:
        """The split, tiles and radix orders the plan uses for length N (and
        the measured times when it was tuned)."""
        c = LengthPlan()
        check(load().fif_plan_length_plan(self._h, int(N), ctypes.byref(c)))
        return c.to_dict()

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

    def set_proposal(self, model: "Model | None") -> None:
        """Let `model` propose m in later runs (None: plain search)."""
        check(load().fif_plan_set_proposal(self._h, model._h if model is not None else None))
        self._model = model      # keep it alive while the plan may use it

    def record_features(self, feats) -> None:
        """Record network inputs of later runs into `feats` (torch bfloat16,
        [B * max_imfs, 1024, 8], row b * max_imfs + j), or stop (None)."""
        torch = _torch()
        if feats is not None:
            shape = (self.B * self.max_imfs, NET_FEATURES, NET_CHANNELS)
            if feats.dtype != torch.bfloat16 or tuple(feats.shape) != shape or not feats.is_cuda \
                    or not feats.is_contiguous():
                raise ValueError("feats must be a contiguous CUDA bfloat16 tensor of shape %s" % (shape,))
        check(load().fif_plan_record_features(self._h, _ptr(feats) if feats is not None else None))
        self._rec = feats

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

    def run(self, signals, delta: float, out: BatchResult | None = None, with_info: bool = True,
            graph: bool = False) -> BatchResult:
        """Enqueue the batched decomposition on the current stream (async);
        graph=True replays it from a captured HIP graph (not on the null
        stream)."""
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
        if graph:
            fn = lib.fif_decompose_batched_graph if signals.dtype == torch.float32 \
                else lib.fif_decompose_batched_graph_f64
        check(fn(self._h, _ptr(signals), float(delta), _ptr(out.imfs), _ptr(out.remainders), _ptr(out.n_imfs),
                 _ptr(out.info_raw) if with_info else 0, _ptr(out.sig_status), aligned, _stream_ptr(torch)))
        return out


    def run_static(self, signals, delta: float, out: BatchResult | None = None,
                   with_info: bool = True) -> BatchResult:
        """fif_decompose_batched_static: the batched decomposition with the
        library's static workspace (no allocation inside the call; FP32;
        plans needing more than STATIC_WORKSPACE_BYTES are refused)."""
        torch = _torch()
        lib = load()
        if signals.dtype != torch.float32 or signals.dim() != 1 or signals.numel() != self.total \
                or not signals.is_cuda or not signals.is_contiguous():
            raise ValueError("signals must be a contiguous 1-D CUDA float32 tensor of %d samples" % self.total)
        if out is None:
            out = self.alloc_outputs(signals.dtype)
        check(lib.fif_decompose_batched_static(self._h, _ptr(signals), float(delta), _ptr(out.imfs),
                                               _ptr(out.remainders), _ptr(out.n_imfs),
                                               _ptr(out.info_raw) if with_info else 0, _ptr(out.sig_status),
                                               _stream_ptr(torch)))
        return out


def tune_cache_lookup(path: str, device_key: str, N: int) -> dict | None:
    """The cached choice for (device_key, N) in the tune cache file, or None."""
    from ._binding import FIF_ERR_NOT_FOUND
    c = LengthPlan()
    st = load().fif_tune_cache_lookup(path.encode(), device_key.encode(), int(N), ctypes.byref(c))
    if st == FIF_ERR_NOT_FOUND:
        return None
    check(st)
    return c.to_dict()


def tune_cache_store(path: str, device_key: str, choice: dict) -> None:
    check(load().fif_tune_cache_store(path.encode(), device_key.encode(), ctypes.byref(LengthPlan.from_dict(choice))))


def device_tune_key() -> str:
    buf = ctypes.create_string_buffer(256)
    check(load().fif_device_tune_key(buf, 256))
    return buf.value.decode()


def release_cache() -> None:
    load().fif_release_cache()


class Model:
    """Step-count proposal network (fif_model_*), parameters as FP32 numpy.

    Inputs are torch bfloat16 CUDA tensors [B, 1024, 8]; targets FP32
    [B, 2] = (log2(m)/16, log2(L)/16).
    """

    def __init__(self, params=None, max_batch: int = 256, path: str | None = None):
        lib = load()
        h = ctypes.c_void_p()
        if path is not None:
            check(lib.fif_model_load(ctypes.byref(h), path.encode(), int(max_batch)))
        else:
            arr = None
            if params is not None:
                p = np.ascontiguousarray(params, dtype=np.float32)
                if p.size != NET_PARAMS:
                    raise ValueError("expected %d parameters" % NET_PARAMS)
                arr = p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
            check(lib.fif_model_create(ctypes.byref(h), arr, int(max_batch)))
        self._h = h.value
        self.max_batch = int(max_batch)

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                load().fif_model_free(self._h)
                self._h = None
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.empty(NET_PARAMS, dtype=np.float32)
        check(load().fif_model_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def set_params(self, params) -> None:
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != NET_PARAMS:
            raise ValueError("expected %d parameters" % NET_PARAMS)
        check(load().fif_model_set_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def save(self, path: str) -> None:
        check(load().fif_model_save(self._h, path.encode()))

    def _check_feats(self, feats):
        torch = _torch()
        if feats.dtype != torch.bfloat16 or feats.dim() != 3 or tuple(feats.shape[1:]) != (NET_FEATURES, NET_CHANNELS) \
                or not feats.is_cuda or not feats.is_contiguous():
            raise ValueError("feats must be a contiguous CUDA bfloat16 tensor [B, %d, %d]" % (NET_FEATURES, NET_CHANNELS))
        return int(feats.shape[0])

    def forward(self, feats):
        torch = _torch()
        B = self._check_feats(feats)
        out = torch.empty(B, 2, dtype=torch.float32, device=feats.device)
        check(load().fif_model_forward(self._h, _ptr(feats), B, _ptr(out), _stream_ptr(torch)))
        return out

    def _targets(self, targets, B):
        torch = _torch()
        if targets.dtype != torch.float32 or tuple(targets.shape) != (B, 2) or not targets.is_cuda \
                or not targets.is_contiguous():
            raise ValueError("targets must be a contiguous CUDA float32 tensor [B, 2]")

    def grad(self, feats, targets):
        """(loss, gradient) of one batch, both torch FP32 CUDA tensors."""
        torch = _torch()
        B = self._check_feats(feats)
        self._targets(targets, B)
        g = torch.empty(NET_PARAMS, dtype=torch.float32, device=feats.device)
        loss = torch.empty(1, dtype=torch.float32, device=feats.device)
        check(load().fif_model_grad(self._h, _ptr(feats), _ptr(targets), B, _ptr(g), _ptr(loss),
                                    _stream_ptr(torch)))
        return loss, g

    def train_step(self, feats, targets, lr: float, loss=None):
        """One Adam step; writes the batch loss into `loss` (FP32 [1]) if given."""
        torch = _torch()
        B = self._check_feats(feats)
        self._targets(targets, B)
        check(load().fif_model_train_step(self._h, _ptr(feats), _ptr(targets), B, float(lr), _ptr(loss),
                                          _stream_ptr(torch)))
