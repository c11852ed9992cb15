"""Seeded synthetic input generators.

This module is shared by the tests, the benchmark and the golden-value
scripts.  It holds no part of the decomposition method: only signal
synthesis (sums of amplitude-modulated tones and chirps plus noise) and the
choice of signal lengths.  Every draw comes from
``numpy.random.default_rng(SeedSequence([workload_id, index]))``.

The paper ships no dataset; these workloads stand in for the
"non-stationary signals" it targets.  Samples sit on the periodic grid
x_i = i/N of [0, 1).  Noise variance for a target SNR (dB) is
mean(s^2) / 10^(SNR/10).
"""
from __future__ import annotations

import bisect
import functools
import math

import numpy as np

# workload ids used in the seed sequences
W_TONES3 = 1      # single FP64 signal, N=4096, three AM tones (8, 40, 200 cycles)
W_CHIRPS = 2      # batch of N=65536 signals, 2-6 AM chirps, 30 dB white noise
W_UNEVEN = 3      # uneven 7-smooth lengths in [1024, 262144], three AM tones
W_LONG = 4        # one N=2^24 signal, 10 drifting tones, 20 dB pink noise
W_TRAIN = 5       # three AM tones at random frequencies, N=65536


def rng_for(workload: int, index: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(workload), int(index)]))


def grid(N: int) -> np.ndarray:
    return np.arange(N, dtype=np.float64) / N


def _add_white_noise(s: np.ndarray, rng: np.random.Generator, snr_db: float) -> np.ndarray:
    p = float(np.mean(s * s))
    sigma = math.sqrt(p / 10.0 ** (snr_db / 10.0))
    return s + sigma * rng.standard_normal(s.size)


def tones3(N: int = 4096, seed_index: int = 1, freqs=(8.0, 40.0, 200.0),
           am_depth: float = 0.3, signs=(1.0, -1.0, 1.0), noise_sigma: float = 0.01,
           workload: int = W_TONES3) -> np.ndarray:
    """Sum of three tones a_i(x) cos(2 pi f_i x), a_i = 1 + depth*sign_i*sin(2 pi x),
    plus N(0, noise_sigma^2) noise.  FP64."""
    x = grid(N)
    s = np.zeros(N)
    for f, sg in zip(freqs, signs):
        a = 1.0 + am_depth * sg * np.sin(2 * np.pi * x)
        s += a * np.cos(2 * np.pi * f * x)
    rng = rng_for(workload, seed_index)
    if noise_sigma > 0:
        s = s + noise_sigma * rng.standard_normal(N)
    return s


def chirps(index: int, N: int = 65536, snr_db: float = 30.0) -> np.ndarray:
    """2-6 amplitude-modulated linear chirps, start frequency log-uniform in
    [4, N/8] cycles, sweep uniform within +-20 % of it (clipped to [4, N/8]),
    AM depth U[0, 0.5] at 1-3 cycles, random phases, white noise at snr_db."""
    rng = rng_for(W_CHIRPS, index)
    x = grid(N)
    nc = int(rng.integers(2, 7))
    fmin, fmax = 4.0, N / 8.0
    s = np.zeros(N)
    for _ in range(nc):
        f0 = math.exp(rng.uniform(math.log(fmin), math.log(fmax)))
        f1 = min(max(f0 * (1.0 + rng.uniform(-0.2, 0.2)), fmin), fmax)
        phi = rng.uniform(0, 2 * np.pi)
        d = rng.uniform(0.0, 0.5)
        u = int(rng.integers(1, 4))
        psi = rng.uniform(0, 2 * np.pi)
        phase = 2 * np.pi * (f0 * x + 0.5 * (f1 - f0) * x * x) + phi
        a = 1.0 + d * np.sin(2 * np.pi * u * x + psi)
        s += a * np.cos(phase)
    return _add_white_noise(s, rng, snr_db)


@functools.lru_cache(maxsize=None)
def smooth7_numbers(limit: int = 1 << 25) -> tuple:
    """Sorted integers <= limit whose prime factors are all <= 7."""
    out = []
    p2 = 1
    while p2 <= limit:
        p3 = p2
        while p3 <= limit:
            p5 = p3
            while p5 <= limit:
                p7 = p5
                while p7 <= limit:
                    out.append(p7)
                    p7 *= 7
                p5 *= 5
            p3 *= 3
        p2 *= 2
    return tuple(sorted(out))


def nearest_smooth7(n: float) -> int:
    """Nearest 7-smooth integer to n; ties go to the smaller one."""
    vals = smooth7_numbers()
    i = bisect.bisect_left(vals, n)
    cands = [vals[j] for j in (i - 1, i) if 0 <= j < len(vals)]
    return min(cands, key=lambda v: (abs(v - n), v))


def uneven_lengths(B: int = 4096, lo: int = 1024, hi: int = 262144) -> np.ndarray:
    """B lengths drawn log-uniform in [lo, hi], rounded to the nearest 7-smooth integer."""
    rng = rng_for(W_UNEVEN, 10**9)
    raw = np.exp(rng.uniform(math.log(lo), math.log(hi), size=B))
    return np.array([nearest_smooth7(v) for v in raw], dtype=np.int64)


def uneven_signal(index: int, N: int) -> np.ndarray:
    """The three-tone generator at length N with a per-signal noise seed."""
    return tones3(N=N, seed_index=index, workload=W_UNEVEN)


def long_drift(N: int = 1 << 24, n_comp: int = 10, snr_db: float = 20.0) -> np.ndarray:
    """10 tones at integer frequencies geometric from 2 to N/16 cycles, each
    with a periodic +-20 % frequency drift, plus pink (1/f power) noise at snr_db."""
    rng = rng_for(W_LONG, 0)
    x = grid(N)
    s = np.zeros(N)
    for i in range(n_comp):
        f = float(round(2.0 * (N / 32.0) ** (i / (n_comp - 1))))
        phi = rng.uniform(0, 2 * np.pi)
        th = rng.uniform(0, 2 * np.pi)
        # instantaneous frequency f (1 + 0.2 sin(2 pi x + phi)); phase periodic on [0,1)
        phase = 2 * np.pi * f * x - (0.2 * f) * (np.cos(2 * np.pi * x + phi) - math.cos(phi)) + th
        s += np.cos(phase)
    white = rng.standard_normal(N)
    W = np.fft.rfft(white)
    j = np.arange(W.size, dtype=np.float64)
    j[0] = 1.0
    W = W / np.sqrt(j)
    W[0] = 0.0
    pink = np.fft.irfft(W, n=N)
    p_sig = float(np.mean(s * s))
    p_n = float(np.mean(pink * pink))
    pink *= math.sqrt(p_sig / 10.0 ** (snr_db / 10.0) / p_n)
    return s + pink


def train_signal(index: int, N: int = 65536) -> np.ndarray:
    """Three AM tones, frequencies log-uniform in [4, N/8], AM depth 0.3 with a
    random sign, N(0, 0.01^2) noise."""
    rng = rng_for(W_TRAIN, index)
    x = grid(N)
    s = np.zeros(N)
    for _ in range(3):
        f = math.exp(rng.uniform(math.log(4.0), math.log(N / 8.0)))
        sg = 1.0 if rng.uniform() < 0.5 else -1.0
        a = 1.0 + 0.3 * sg * np.sin(2 * np.pi * x)
        s += a * np.cos(2 * np.pi * f * x + rng.uniform(0, 2 * np.pi))
    return s + 0.01 * rng.standard_normal(N)


def train_params(index: int, N: int = 65536) -> np.ndarray:
    """(frequency, AM sign, phase) of the three tones of train_signal(index)."""
    rng = rng_for(W_TRAIN, index)
    out = np.empty((3, 3))
    for c in range(3):
        out[c, 0] = math.exp(rng.uniform(math.log(4.0), math.log(N / 8.0)))
        out[c, 1] = 1.0 if rng.uniform() < 0.5 else -1.0
        out[c, 2] = rng.uniform(0, 2 * np.pi)
    return out


def train_batch(first: int, count: int, N: int = 65536, device: str = "cuda"):
    """Signals first .. first+count-1 of the train_signal family synthesised on
    the device (torch, FP64 then rounded to FP32): the same tones as
    train_signal, with N(0, 0.01^2) noise from a torch generator seeded with
    (W_TRAIN, first) instead of numpy's stream.  Returns [count, N] FP32."""
    import torch
    P = torch.tensor(np.stack([train_params(first + i, N) for i in range(count)]), dtype=torch.float64,
                     device=device)                                   # [count, 3, 3]
    x = torch.arange(N, dtype=torch.float64, device=device) / N
    two_pi = 2.0 * math.pi
    am = torch.sin(two_pi * x)                                        # [N]
    s = torch.zeros(count, N, dtype=torch.float64, device=device)
    for c in range(3):
        f, sg, ph = P[:, c, 0:1], P[:, c, 1:2], P[:, c, 2:3]
        s += (1.0 + 0.3 * sg * am) * torch.cos(two_pi * f * x + ph)
    g = torch.Generator(device=device)
    g.manual_seed(int(np.random.SeedSequence([W_TRAIN, int(first)]).generate_state(1)[0]))
    s += 0.01 * torch.randn(count, N, dtype=torch.float64, device=device, generator=g)
    return s.to(torch.float32)
