"""Training and evaluation of the step-count proposal network on the GPU.

Training data are the method's own decompositions: a plan records the
network input rows of every outer step (fif_plan_record_features) while the
plain decomposition runs, and the selected (m, L) of each IMF are the
targets.  Training runs entirely in the library's BF16 MFMA forward and
backward kernels (fif_model_train_step); Python only draws minibatch
indices.  Signals: three amplitude-modulated tones with log-uniform
frequencies in [4, N/8] cycles, AM depth 0.3 of random sign and N(0, 0.01^2)
noise, N = 65536 (siggen.train_batch).

    python -m paper_1802_01359_amd.proposal train --signals 200000 --out net.fifnet
    python -m paper_1802_01359_amd.proposal eval --model net.fifnet --count 4096
"""
from __future__ import annotations

import argparse
import math
import sys
import time

import numpy as np

from . import IMF_CAP, NET_PARAMS, Model, Plan

N_TRAIN = 65536
DELTA = 1e-3
MAX_IMFS = 8
EVAL_FIRST = 10_000_000     # first signal index of the held-out evaluation set

_KW, _CH = 7, 64


def init_params(seed: int = 0, m_prior: float = 64.0) -> np.ndarray:
    """He-normal convolution weights (the two live input channels of layer 0),
    zero biases, a small head whose bias starts at log2(m_prior)/16."""
    rng = np.random.default_rng(seed)
    out, off = np.zeros(NET_PARAMS, dtype=np.float32), 0
    for l in range(6):
        cin = 8 if l == 0 else _CH
        live = 2 if l == 0 else _CH
        W = np.zeros((_KW, cin, _CH))
        W[:, :live, :] = rng.normal(0.0, math.sqrt(2.0 / (_KW * live)), (_KW, live, _CH))
        out[off:off + W.size] = W.ravel()
        off += W.size + _CH
    out[off:off + 2 * _CH] = rng.normal(0.0, 0.01, 2 * _CH)
    out[off + 2 * _CH] = math.log2(m_prior) / 16.0
    out[off + 2 * _CH + 1] = math.log2(16.0) / 16.0
    assert off + 2 * _CH + 2 == NET_PARAMS
    return out


def _torch():
    import torch
    return torch


class Recorder:
    """A plan over `count` signals of length N that records network inputs."""

    def __init__(self, count: int, N: int = N_TRAIN, max_imfs: int = MAX_IMFS):
        torch = _torch()
        self.count, self.N, self.max_imfs = count, N, max_imfs
        self.plan = Plan([N] * count, max_imfs)
        self.feats = torch.zeros(count * max_imfs, 1024, 8, dtype=torch.bfloat16, device="cuda")
        self.plan.record_features(self.feats)
        self.out = self.plan.alloc_outputs(torch.float32)

    def run(self, x, delta: float = DELTA):
        """Decompose x ([count, N] FP32 on the device); returns (rows, targets):
        indices of the valid records and their FP32 targets on the device."""
        torch = _torch()
        self.plan.run(x.reshape(-1), delta, out=self.out)
        info = self.out.info()
        n = self.out.n_imfs.cpu().numpy()
        j = np.arange(self.max_imfs)[None, :]
        ok = (j < n[:, None]) & ((info["flags"] & IMF_CAP) == 0)
        rows = np.flatnonzero(ok.ravel())
        m = info["m"].ravel()[rows].astype(np.float64)
        L = info["L"].ravel()[rows].astype(np.float64)
        tg = np.stack([np.log2(m) / 16.0, np.log2(L) / 16.0], axis=1).astype(np.float32)
        return rows, torch.tensor(tg, device="cuda"), info


def train(signals: int, chunk: int = 1024, batch: int = 256, epochs: int = 1, lr: float = 1e-3,
          seed: int = 0, params=None, log=print) -> Model:
    """Train on `signals` decompositions (signal indices 0 .. signals-1)."""
    import siggen
    torch = _torch()
    model = Model(init_params(seed) if params is None else params, max_batch=batch)
    rec = Recorder(chunk)
    rng = np.random.default_rng(seed)
    n_chunks = max(1, signals // chunk)
    total_steps = 0
    # records per chunk: about MAX_IMFS per signal
    est_steps = epochs * n_chunks * max(1, (chunk * MAX_IMFS) // batch)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    t0 = time.time()
    step = 0
    for ep in range(epochs):
        ep_loss, ep_n = 0.0, 0
        for c in range(n_chunks):
            x = siggen.train_batch(c * chunk, chunk, N_TRAIN)
            rows, tg, _ = rec.run(x)
            perm = rng.permutation(rows.size)
            for b0 in range(0, rows.size - batch + 1, batch):
                sel = perm[b0:b0 + batch]
                idx = torch.tensor(rows[sel], device="cuda")
                f = rec.feats.index_select(0, idx).contiguous()
                t = tg.index_select(0, torch.tensor(sel, device="cuda")).contiguous()
                # cosine decay to lr/100
                frac = min(1.0, step / max(1, est_steps))
                lr_t = lr * (0.01 + 0.99 * 0.5 * (1.0 + math.cos(math.pi * frac)))
                model.train_step(f, t, lr_t, loss)
                step += 1
                if step % 64 == 0:
                    ep_loss += float(loss.cpu()[0])
                    ep_n += 1
            total_steps = step
            if (c + 1) % max(1, n_chunks // 10) == 0 or c + 1 == n_chunks:
                log("epoch %d chunk %d/%d steps %d loss %.3g (%.1f s)" % (
                    ep, c + 1, n_chunks, total_steps, ep_loss / max(ep_n, 1), time.time() - t0))
                ep_loss, ep_n = 0.0, 0
    torch.cuda.synchronize()
    return model


def evaluate(model: Model | None, first: int = EVAL_FIRST, count: int = 4096, delta: float = DELTA,
             max_imfs: int = MAX_IMFS, repeats: int = 3) -> dict:
    """Decompose a held-out batch without and with the proposal; check that
    both give the same decomposition; report search work and times."""
    import siggen
    torch = _torch()
    x = siggen.train_batch(first, count, N_TRAIN).reshape(-1)
    plan = Plan([N_TRAIN] * count, max_imfs)
    res = {}
    outs = {}
    for mode in ("plain", "proposal"):
        plan.set_proposal(model if mode == "proposal" else None)
        out = plan.alloc_outputs(torch.float32)
        plan.run(x, delta, out=out)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(repeats):
            plan.run(x, delta, out=out)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / repeats
        info = out.info()
        n = out.n_imfs.cpu().numpy()
        valid = np.arange(max_imfs)[None, :] < n[:, None]
        ev32 = (info["evals"] & 0xFFFF)[valid].astype(np.float64)
        ev64 = (info["evals"] >> 16)[valid].astype(np.float64)
        res[mode] = dict(ms_per_batch=ms, samples_per_s=count * N_TRAIN / (ms * 1e-3),
                         fp32_passes_per_imf=float(ev32.mean()), fp64_evals_per_imf=float(ev64.mean()),
                         imfs=int(valid.sum()))
        outs[mode] = (out, info, n)
    plan.set_proposal(None)
    (o0, i0, n0), (o1, i1, n1) = outs["plain"], outs["proposal"]
    same = bool(np.array_equal(n0, n1) and all(np.array_equal(i0[k], i1[k]) for k in ("k", "L", "m", "sd", "sd_prev"))
                and torch.equal(o0.imfs, o1.imfs) and torch.equal(o0.remainders, o1.remainders))
    res["identical"] = same
    if model is not None:
        # proposal accuracy on the same records
        rec = Recorder(min(count, 1024))
        rows, tg, info = rec.run(x[:rec.count * N_TRAIN].reshape(rec.count, N_TRAIN), delta)
        ys = []
        for b0 in range(0, rows.size, model.max_batch):
            idx = torch.tensor(rows[b0:b0 + model.max_batch], device="cuda")
            ys.append(model.forward(rec.feats.index_select(0, idx).contiguous()))
        y = torch.cat(ys).cpu().numpy().astype(np.float64)
        t = tg.cpu().numpy().astype(np.float64)
        err = np.abs(y[:, 0] - t[:, 0]) * 16.0
        m_hat = np.clip(np.rint(2.0 ** (16.0 * y[:, 0])), 1, None)
        m = np.rint(2.0 ** (16.0 * t[:, 0]))
        res["log2_m_abs_err_mean"] = float(err.mean())
        res["log2_m_abs_err_p90"] = float(np.quantile(err, 0.9))
        res["m_exact_rate"] = float(np.mean(m_hat == m))
    return res


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--signals", type=int, default=200_000)
    t.add_argument("--chunk", type=int, default=1024)
    t.add_argument("--batch", type=int, default=256)
    t.add_argument("--epochs", type=int, default=1)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--out", required=True)
    t.add_argument("--eval-count", type=int, default=1024)
    e = sub.add_parser("eval")
    e.add_argument("--model", required=True)
    e.add_argument("--count", type=int, default=4096)
    a = ap.parse_args(argv)
    log = lambda *s: print(*s, file=sys.stderr, flush=True)  # noqa: E731
    if a.cmd == "train":
        model = train(a.signals, a.chunk, a.batch, a.epochs, a.lr, a.seed, log=log)
        model.save(a.out)
        log("saved", a.out)
        if a.eval_count:
            log(evaluate(model, count=a.eval_count))
    else:
        model = Model(path=a.model, max_batch=1024)
        print(evaluate(model, count=a.count))
    return 0


if __name__ == "__main__":
    sys.exit(main())
