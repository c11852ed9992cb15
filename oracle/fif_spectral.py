"""FP64 CPU reference of the paper's direct (FFT) form of DIF.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).

Section 4 of the paper turns each inner loop into one step: with periodic
extension W is circulant, its eigenvalues are the DFT of its first column
(equation "Lambdas"), and (I - W)^{N0} s = IDFT((1 - lambda)^{N0} DFT(s))
(Theorem 5, equation "IMF1_direct", and equation "One step_algo").  The
number of steps is found, as Section 4 describes, by trying N0 = 1, 2, 3, ...
and stopping at the first one whose SD is <= delta; SD is evaluated from the
spectrum by Parseval's identity (the step used in the proof of Theorem 2).

Everything else (extrema count, mask length, rounding floor, window column)
follows the same readings as the time-domain oracle and reuses its helpers.
numpy's FFT is the only library primitive.
"""
from __future__ import annotations

import math

import numpy as np

from . import dif


def eigenvalues(N: int, L: int) -> np.ndarray:
    """lambda_p, p = 0..N-1: DFT of the circulant's first column (eq. "Lambdas")."""
    c = dif.window_column(N, L)
    return np.fft.fft(c).real


def decompose(s, delta: float, max_imfs: int, *, mask_rule: int = 0, nu: float = 1.6,
              max_inner: int = 1_000_000, floor_tau: float = 1e-9) -> dif.Decomposition:
    s = np.ascontiguousarray(np.asarray(s, dtype=np.float64))
    N = s.size
    r = s.copy()
    maxs = float(np.max(np.abs(s))) if N else 0.0
    imfs = []
    out = dif.Decomposition(imfs=np.zeros((0, N)), remainder=r)
    reason = dif.STOP_MAX_IMFS
    for _ in range(max_imfs):
        mean = math.fsum(r) / N
        dev = float(np.max(np.abs(r - mean)))
        thr = floor_tau * maxs
        if dev <= thr:
            reason = dif.STOP_FLOOR
            break
        k, margin = dif.count_extrema(r)
        if k < 2:
            reason = dif.STOP_FEW_EXTREMA
            break
        L = dif.mask_length(N, k, mask_rule, nu)
        lam = eigenvalues(N, L)
        R = np.fft.fft(r)
        P = (R.real * R.real + R.imag * R.imag)
        mu = (1.0 - lam) ** 2
        lam2 = lam * lam
        # N0 = 1, 2, ...: SD_{N0} = ||(1-lam)^{N0-1} lam R|| / ||(1-lam)^{N0-1} R||
        x = P.copy()
        m = 0
        sd = 0.0
        sd_prev = math.inf
        flags = 0
        while True:
            m += 1
            num = float(np.sum(x * lam2))
            den = float(np.sum(x))
            sd_prev = sd if m > 1 else math.inf
            sd = math.sqrt(num / den) if den > 0 else 0.0
            if sd <= delta:
                break
            if m >= max_inner:
                flags |= dif.FLAG_CAP
                break
            x = x * mu
        g = np.power(1.0 - lam, m)
        imf = np.fft.ifft(g * R).real
        imfs.append(imf)
        r = r - imf
        out.k.append(k)
        out.L.append(L)
        out.m.append(m)
        out.sd.append(sd)
        out.sd_prev.append(sd_prev)
        out.margin_k.append(margin)
        out.floor_ratio.append(dev / thr if thr > 0 else math.inf)
        out.flags.append(flags)
    out.imfs = np.array(imfs) if imfs else np.zeros((0, N))
    out.remainder = r
    out.stop_reason = reason
    return out
