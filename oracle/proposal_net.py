"""FP64 CPU reference of the step-count proposal network and its features.

TEST INFRASTRUCTURE ONLY: the GPU kernels of the learned proposal are checked
against these functions (forward outputs, loss, every parameter gradient).
Nothing here is shared with, or imported by, the GPU library.

The network is not part of the paper.  It proposes, for each IMF, the inner
step count m that the Section 4 scan (SD <= delta, equation "SD") would
select, from the residual's power spectrum and the mask length L; the exact
scan then confirms or corrects the proposal, so the decomposition itself is
unchanged.  Definition (all "conv" layers: kernel 7, stride 2, zero padding
3, 64 output channels, ReLU):

    input   x[b, p, c], p < 1024 positions, c < 8 channels (channel 0: log
            power spectrum, channel 1: log2(L)/16, channels 2..7: zero)
    conv_l  z[b, q, o] = bias_l[o] + sum_{t<7, c} W_l[t, c, o] * a[b, 2q+t-3, c]
            (a = 0 outside 0 <= 2q+t-3 < length), a' = max(z, 0);
            six layers, lengths 1024 -> 512 -> 256 -> 128 -> 64 -> 32 -> 16
    head    h[b, o] = mean_q a6[b, q, o];  y[b, u] = bh[u] + sum_o Wh[u, o] h[b, o]
    loss    sum_{b,u} (y[b, u] - target[b, u])^2 / (2 B)

Targets are log2(m)/16 and log2(L)/16.  Flat parameter order: for each conv
layer W_l [7][C_in][64] then bias_l [64] (C_in = 8 for the first layer, 64
after), then Wh [2][64], bh [2].

With ``bf16=True`` the reference rounds, like the GPU kernels, the stored
activations, the conv weights and the backpropagated pre-activation
gradients to bfloat16 (round to nearest even); every other operation is
FP64.  numpy matmuls (einsum) are the only library primitive.
"""
from __future__ import annotations

import numpy as np

NFEAT = 1024
CIN0 = 8
CH = 64
KW = 7
PAD = 3
STRIDE = 2
NLAYERS = 6
NOUT = 2


def layer_shapes():
    """(C_in, length in, length out) of each conv layer."""
    out, cin, n = [], CIN0, NFEAT
    for _ in range(NLAYERS):
        out.append((cin, n, n // 2))
        cin, n = CH, n // 2
    return out


def param_layout():
    """List of (name, shape, offset) in flat parameter order."""
    lay, off = [], 0
    for l, (cin, _, _) in enumerate(layer_shapes()):
        for name, shape in ((f"W{l}", (KW, cin, CH)), (f"b{l}", (CH,))):
            lay.append((name, shape, off))
            off += int(np.prod(shape))
    for name, shape in (("Wh", (NOUT, CH)), ("bh", (NOUT,))):
        lay.append((name, shape, off))
        off += int(np.prod(shape))
    return lay


def n_params() -> int:
    name, shape, off = param_layout()[-1]
    return off + int(np.prod(shape))


def unpack(flat):
    flat = np.asarray(flat, dtype=np.float64)
    return {name: flat[off:off + int(np.prod(shape))].reshape(shape) for name, shape, off in param_layout()}


def pack(d) -> np.ndarray:
    out = np.zeros(n_params())
    for name, shape, off in param_layout():
        out[off:off + int(np.prod(shape))] = np.asarray(d[name], dtype=np.float64).reshape(-1)
    return out


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even) via FP32, returned as FP64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _im2col(a, lout):
    """cols[b, q, t, c] = a[b, 2q + t - 3, c] (zero outside)."""
    B, n, c = a.shape
    ap = np.zeros((B, n + 2 * PAD + 1, c))
    ap[:, PAD:PAD + n] = a
    cols = np.empty((B, lout, KW, c))
    for t in range(KW):
        cols[:, :, t, :] = ap[:, t:t + STRIDE * lout:STRIDE, :]
    return cols


def forward(flat, x, bf16: bool = False):
    """Outputs y [B, 2] and the cache backward() needs."""
    P = unpack(flat)
    r = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    a = r(np.asarray(x, dtype=np.float64))
    cache = []
    for l, (cin, n, lout) in enumerate(layer_shapes()):
        W = r(P[f"W{l}"])
        cols = _im2col(a, lout)
        z = np.einsum("bqtc,tco->bqo", cols, W) + P[f"b{l}"]
        a = r(np.maximum(z, 0.0))
        cache.append((cols, W, a))
    h = a.mean(axis=1)
    y = h @ P["Wh"].T + P["bh"]
    return y, (cache, h)


def loss_and_grad(flat, x, target, bf16: bool = False):
    """Loss and the flat gradient of every parameter."""
    P = unpack(flat)
    r = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    target = np.asarray(target, dtype=np.float64)
    y, (cache, h) = forward(flat, x, bf16)
    B = y.shape[0]
    diff = y - target
    loss = float(np.sum(diff * diff) / (2 * B))
    dy = diff / B
    g = {"Wh": dy.T @ h, "bh": dy.sum(axis=0)}
    dh = dy @ P["Wh"]
    lout_last = cache[-1][2].shape[1]
    da = np.repeat(dh[:, None, :] / lout_last, lout_last, axis=1)
    for l in range(NLAYERS - 1, -1, -1):
        cols, W, a = cache[l]
        dz = r(da * (a > 0))
        g[f"W{l}"] = np.einsum("bqtc,bqo->tco", cols, dz)
        g[f"b{l}"] = dz.sum(axis=(0, 1))
        if l == 0:
            break
        dcols = np.einsum("bqo,tco->bqtc", dz, W)
        cin, n, lout = layer_shapes()[l]
        dap = np.zeros((dz.shape[0], n + 2 * PAD + 1, cin))
        for t in range(KW):
            dap[:, t:t + STRIDE * lout:STRIDE, :] += dcols[:, :, t, :]
        da = dap[:, PAD:PAD + n]
    return loss, pack(g)


def features(spectrum, L: int) -> np.ndarray:
    """Input rows [1024, 8] of one residual from its half spectrum R[0..N/2].

    Group q covers bins 1 + floor(q H / 1024) <= j < 1 + floor((q+1) H / 1024)
    (H = N/2; a group that would be empty takes its first bin alone); channel
    0 is log2(mean power of the group / total power + 2^-60) / 16, channel 1
    is log2(L) / 16.  The DC bin is left out (it never enters an IMF).
    """
    R = np.asarray(spectrum)
    H = R.size - 1
    pw = np.abs(R[1:]) ** 2
    tot = float(pw.sum())
    out = np.zeros((NFEAT, CIN0))
    for q in range(NFEAT):
        j0 = (q * H) // NFEAT
        j1 = max(((q + 1) * H) // NFEAT, j0 + 1)
        mean = float(pw[j0:j1].mean())
        out[q, 0] = np.log2(mean / tot + 2.0 ** -60) / 16.0 if tot > 0 else -60.0 / 16.0
    out[:, 1] = np.log2(float(L)) / 16.0
    return out
