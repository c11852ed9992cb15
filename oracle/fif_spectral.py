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

Variants beyond the plain method (each off by default):
  - stop="abs": the absolute criterion of equation "Discrete_Abs_StopCond",
    ||s_{m+1} - s_m||_2 < delta, IMF = s_m (m >= 1, the smallest such m);
  - stop="apriori": m = N0, the smallest N0 >= 1 satisfying inequality
    "N0_discrete" of Theorem 5, no scan at all (the a-priori estimate the
    paper's Section 4 mentions before the SD scan);
  - gamma > 0: the thresholded IMF of equation "IMF_cont_stop_threshold",
    discretised: a bin whose factor (1 - lambda_j)^m is >= 1 - gamma is taken
    whole (lambda_j replaced by 0);
  - mask_rule=2: the spectral-peak mask length of Section 2 ("highest
    frequency peak" of the spectrum), read as L = ceil(N / f), f the highest
    bin 1 <= f <= N/2 whose power is >= peak_rho times the strongest
    non-constant bin's (a pure tone at f cycles then gets the L of rule 0);

SD with the relative criterion (the default) is a weighted mean of lambda^2
over the bins the residual holds, with weights P_j mu_j^(m-1).  Two readings
keep it what exact arithmetic gives once m is large (the paper is silent):
bins with |R_j|^2 < SD_NOISE max_{j>=1} |R_j|^2 are rounding noise of exact
zeros (an FP64 FFT resolves R to ~1e-16 of its largest bin) and are left out
of the sums; and the sums are taken scale-free, every weight divided by the
largest, so that they never underflow.  Without either, a pure tone whose
lambda exceeds delta (SD constant, the case the iteration cap exists for)
would stop wherever the tone's power underflows or the noise takes over.
  - window=shape: another window than the triangle of equation "triangular".  Section
    4 only needs W's eigenvalues, the DFT of its first column (equation
    "Lambdas"), which can be tabulated for any filter.  Read here as: h, the
    non-negative samples `shape` (at x = i/K, i = 0..K) linearly
    interpolated at x = |q|/L for |q| <= L - 1; the window is h convolved
    with itself, divided by (sum h)^2 so that it sums to 1 (for shape
    [1, 0], h is the triangle and the window is the default one); its taps
    are folded modulo N into the circulant's first column.  The window is
    symmetric and its DFT is (DFT h)^2 (convolution theorem), so every
    eigenvalue lies in [0, 1]; they are computed in that form, as
    (H_j / H_0)^2 with H the DFT of the folded h.  Reading where the paper is
    silent: |H_j / H_0| < 1e-13 is taken as an exact zero (an FP64 FFT
    resolves H only to ~1e-15, so the exact zeros a window spectrum can have,
    such as a box's, would otherwise come out as rounding noise whose size
    decides how the SD of later steps ends).
"""
from __future__ import annotations

import math

import numpy as np

from . import dif


def eigenvalues(N: int, L: int) -> np.ndarray:
    """lambda_p, p = 0..N-1: DFT of the circulant's first column (eq. "Lambdas")."""
    c = dif.window_column(N, L)
    return np.fft.fft(c).real


def eigenvalues_closed(N: int, L: int) -> np.ndarray:
    """lambda_p, p = 0..N-1, from the closed form of equation "eig2":
    [sin(pi L p / N) / (L sin(pi p / N))]^4, lambda_0 = 1, with L p reduced
    modulo N exactly and folded to min(t, N - t) (the fourth power hides the
    sign) so that every sine argument is at most pi/2: relative, not
    absolute, rounding error, which matters once m ~ 1e5 multiplies it."""
    p = np.arange(N, dtype=np.int64)
    t = ((L % N) * p) % N
    t = np.minimum(t, N - t)
    u = np.minimum(p, N - p)
    lam = np.ones(N)
    nz = p != 0
    q = np.sin(np.pi * t[nz] / N) / (L * np.sin(np.pi * u[nz] / N))
    lam[nz] = q ** 4
    return lam


def shape_taps(L: int, shape) -> np.ndarray:
    """h_q for q = -(L-1) .. L-1 (unnormalised): the shape's samples at
    x_i = i/K, i = 0..K, linearly interpolated at x = |q|/L; the position
    |q| K / L is split exactly into an integer part and a remainder."""
    shape = np.asarray(shape, dtype=np.float64)
    K = shape.size - 1
    q = np.arange(-(L - 1), L, dtype=np.int64)
    u = np.abs(q) * K
    i = u // L
    rr = u % L
    return shape[i] + (shape[i + 1] - shape[i]) * (rr.astype(np.float64) / float(L))


def window_column_shape(N: int, L: int, shape) -> np.ndarray:
    """First column of the circulant W of a sampled window shape: the taps of
    h * h / (sum h)^2 (q = -(2L-2) .. 2L-2) folded modulo N."""
    h = shape_taps(L, shape)
    w = np.convolve(h, h) / float(np.sum(h)) ** 2
    q = np.arange(-(2 * L - 2), 2 * L - 1, dtype=np.int64)
    c = np.zeros(N)
    np.add.at(c, q % N, w)
    return c


# |H_j / H_0| below this is an exact zero of the window spectrum
WINDOW_ZERO = 1e-13


def eigenvalues_shape(N: int, L: int, shape) -> np.ndarray:
    """lambda_p, p = 0..N-1, of a sampled window shape (equation "Lambdas"
    for the column of window_column_shape, by the convolution theorem):
    (H_p / H_0)^2 with H the DFT of the folded taps h, H_0 = sum h; values of
    |H_p / H_0| below WINDOW_ZERO are exact zeros; lambda_0 = 1."""
    h = shape_taps(L, shape)
    q = np.arange(-(L - 1), L, dtype=np.int64)
    f = np.zeros(N)
    np.add.at(f, q % N, h)
    H = np.fft.fft(f).real / float(np.sum(h))
    lam = np.where(np.abs(H) < WINDOW_ZERO, 0.0, np.minimum(H * H, 1.0))
    lam[0] = 1.0
    return lam


# |R_j|^2 below this fraction of the strongest non-constant bin is not counted in SD
SD_NOISE = 1e-26


def _pow1m(lam, e):
    """(1 - lambda)^e as exp(e log1p(-lambda)): the factor of equation
    "IMF1_direct" without rounding 1 - lambda first (whose relative error
    would grow e-fold); lambda is clamped to [0, 1], where it lies (a fourth
    power, at most 1), so FFT rounding cannot push a factor above 1."""
    lam = np.clip(lam, 0.0, 1.0)
    with np.errstate(divide="ignore"):
        lg = np.log1p(-lam)
    return np.exp(e * lg) if e > 0 else np.ones_like(lam)


def zero_eigenvalues(N: int, L: int) -> int:
    """k of Theorem 5: eigenvalues lambda_p (p = 1..N-1) that are exactly 0,
    i.e. sin(pi L p / N) = 0, i.e. N divides L*p."""
    return sum(1 for p in range(1, N) if (L * p) % N == 0)


def apriori_n0(R, N: int, L: int, delta: float) -> int:
    """Smallest N0 >= 1 with N0^N0 / (N0+1)^(N0+1) < delta / (||U^T r||_inf
    sqrt(N - 1 - k)) (Theorem 5), compared in logarithms; R = DFT(r)."""
    st_inf = float(np.max(np.abs(R))) / math.sqrt(N)   # unitary DFT coefficients
    rest = N - 1 - zero_eigenvalues(N, L)
    if st_inf == 0.0 or rest <= 0:
        return 1
    rhs = math.log(delta / (st_inf * math.sqrt(rest)))

    def lhs(n):
        return n * math.log(n) - (n + 1) * math.log(n + 1)
    hi = 1
    while lhs(hi) >= rhs:
        hi *= 2
    lo = hi // 2   # lhs(lo) >= rhs unless lo == 0
    if lo == 0:
        return 1
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if lhs(mid) < rhs:
            hi = mid
        else:
            lo = mid
    return hi


def peak_frequency(R, rho: float) -> int:
    """Highest bin f in [1, N/2] with |R_f|^2 >= rho * max_{1<=j<=N/2} |R_j|^2."""
    N = R.size
    P = np.abs(R[1:N // 2 + 1]) ** 2
    top = float(P.max()) if P.size else 0.0
    idx = np.flatnonzero(P >= rho * top)
    return int(idx[-1]) + 1 if idx.size and top > 0 else 1


def imfs_at(s, Ls, ms, gamma: float = 0.0):
    """IMFs and remainder of the direct form (Theorem 5, equation
    "IMF1_direct"; Section 4, equation "One step_algo") at given mask
    lengths Ls[j] and step counts ms[j], without the search for m: IMF_j =
    IDFT((1 - lambda)^m_j DFT(r_j)), r_{j+1} = r_j - IMF_j.  The signal is
    real, so the half spectrum (numpy's real FFT) carries the same
    computation at half the cost; it lets a test rebuild long decompositions
    whose decisions were stored."""
    r = np.ascontiguousarray(np.asarray(s, dtype=np.float64)).copy()
    N = r.size
    imfs = []
    for L, m in zip(Ls, ms):
        R = np.fft.rfft(r)
        g = _pow1m(eigenvalues_closed(N, int(L))[:R.size], int(m))
        if gamma > 0.0:
            g = np.where(g >= 1.0 - gamma, 1.0, g)
        imf = np.fft.irfft(g * R, n=N)
        imfs.append(imf)
        r = r - imf
    return (np.array(imfs) if imfs else np.zeros((0, N))), r


def decompose(s, delta: float, max_imfs: int, *, mask_rule: int = 0, nu: float = 1.6,
              max_inner: int = 1_000_000, floor_tau: float = 1e-9, stop: str = "sd",
              gamma: float = 0.0, peak_rho: float = 0.1, search: str = "linear",
              window=None) -> dif.Decomposition:
    if window is not None and stop == "apriori":
        raise ValueError("the a-priori N0 counts the triangle window's zero eigenvalues")
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
        R = np.fft.fft(r)
        if mask_rule == 2:
            L = max(1, -(-N // peak_frequency(R, peak_rho)))
        else:
            L = dif.mask_length(N, k, mask_rule, nu)
        lam = eigenvalues_closed(N, L) if window is None else eigenvalues_shape(N, L, window)
        P = (R.real * R.real + R.imag * R.imag)
        mu = (1.0 - lam) ** 2
        lam2 = lam * lam
        flags = 0
        if stop == "sd":
            # the bins SD counts: the constant one and those above the noise floor
            qmax = float(np.max(P[1:])) if N > 1 else 0.0
            Psd = np.where(P >= SD_NOISE * qmax, P, 0.0)
            Psd[0] = P[0]
        if stop == "sd" and search == "bisect":
            # SD_m is non-increasing in m, so the smallest m with SD_m <= delta
            # is found by doubling then bisection on the same Parseval sums
            live = (Psd > 0.0) & (lam < 1.0)
            with np.errstate(divide="ignore"):
                l1 = np.log1p(-np.clip(lam, 0.0, 1.0))

            def sd_at(mm):
                if mm == 1:
                    num, den = float(np.sum(Psd * lam2)), float(np.sum(Psd))
                else:
                    if not np.any(live):
                        return 0.0
                    a = 2.0 * (mm - 1) * l1[live]
                    x = Psd[live] * np.exp(a - a.max())
                    num, den = float(np.sum(x * lam2[live])), float(np.sum(x))
                return math.sqrt(num / den) if den > 0 else 0.0
            hi = 1
            while sd_at(hi) > delta and hi < max_inner:
                hi = min(max_inner, 2 * hi)
            if sd_at(hi) > delta:
                m = max_inner
                flags |= dif.FLAG_CAP
            else:
                lo = hi // 2 if hi > 1 else 0          # sd_at(lo) > delta (lo = 0: none)
                while hi - lo > 1:
                    mid = (lo + hi) // 2
                    if sd_at(mid) <= delta:
                        hi = mid
                    else:
                        lo = mid
                m = hi
            sd = sd_at(m)
            sd_prev = sd_at(m - 1) if m > 1 else math.inf
        elif stop == "sd":
            # N0 = 1, 2, ...: SD_{N0} = ||(1-lam)^{N0-1} lam R|| / ||(1-lam)^{N0-1} R||,
            # the weights rescaled by their largest after every step
            x = Psd.copy()
            m = 0
            sd = 0.0
            sd_prev = math.inf
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
                top = float(np.max(x))
                if top > 0.0:
                    x = x / top
        elif stop == "abs":
            # ||s_{m+1} - s_m||_2 = ||W s_m||_2 = sqrt(sum |R|^2 lam^2 mu^m / N) (Parseval)
            x = P * mu
            m = 0
            sd = math.sqrt(float(np.sum(P * lam2)) / N)   # m = 0
            while True:
                m += 1
                sd_prev = sd
                sd = math.sqrt(float(np.sum(x * lam2)) / N)
                if sd < delta:
                    break
                if m >= max_inner:
                    flags |= dif.FLAG_CAP
                    break
                x = x * mu
        elif stop == "apriori":
            m = apriori_n0(R, N, L, delta)
            if m > max_inner:
                m = max_inner
                flags |= dif.FLAG_CAP
            sd = math.sqrt(float(np.sum(P * lam2 * _pow1m(lam, 2 * m))) / N)
            sd_prev = math.sqrt(float(np.sum(P * lam2 * _pow1m(lam, 2 * (m - 1)))) / N)
        else:
            raise ValueError(stop)
        g = _pow1m(lam, m)
        if gamma > 0.0:
            g = np.where(g >= 1.0 - gamma, 1.0, g)
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
