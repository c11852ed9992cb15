"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test would fail under a plausible slip in the oracle: a wrong window
normalisation or support (column sums, closed-form spectrum, dense brute
force), a wrong sign or index in the convolution (pure-tone decay, dense
brute force), a wrong stop rule or iteration count (exact rationals,
monotone SD, pure tone with cap), a wrong extrema rule (exhaustive patterns),
or a dropped subtraction in the outer loop (reconstruction, zero means).
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import siggen
from oracle import dif, fif_spectral


# ---------------------------------------------------------------- window ---

def closed_form_lambda(N: int, L: int) -> np.ndarray:
    """[sin(pi L j/N) / (L sin(pi j/N))]^4 with the argument L*j reduced mod N
    in integers (the DFT of the triangle-squared window on the grid)."""
    j = np.arange(N, dtype=np.int64)
    t = (L * j) % N
    t = np.minimum(t, N - t)
    u = np.minimum(j, N - j)
    lam = np.ones(N)
    nz = u != 0
    lam[nz] = (np.sin(np.pi * t[nz] / N) / (L * np.sin(np.pi * u[nz] / N))) ** 4
    return lam


@pytest.mark.parametrize("N,L", [(5, 1), (5, 2), (7, 3), (16, 4), (17, 9), (64, 31), (64, 64),
                                 (64, 130), (100, 7), (4096, 21), (4096, 2048), (99, 200)])
def test_window_column_is_a_filter(N, L):
    c = dif.window_column(N, L)
    assert c.min() >= 0.0
    assert abs(c.sum() - 1.0) < 1e-14
    # symmetric: c_{N-p} = c_p (Definition 2: symmetric filter)
    assert np.allclose(c[1:], c[1:][::-1], rtol=0, atol=1e-17)


@pytest.mark.parametrize("N,L", [(5, 2), (8, 3), (15, 4), (64, 9), (64, 64), (63, 100),
                                 (1024, 21), (4096, 512), (4096, 4096), (3000, 1234)])
def test_window_spectrum_matches_closed_form(N, L):
    lam_fft = fif_spectral.eigenvalues(N, L)
    lam_cf = closed_form_lambda(N, L)
    assert np.max(np.abs(lam_fft - lam_cf)) < 1e-14
    assert lam_cf[0] == 1.0


@pytest.mark.parametrize("N,L", [(9, 2), (16, 5), (31, 7), (48, 12)])
def test_window_spectrum_direct_cosine_sum(N, L):
    """lambda_j = c_0 + sum_k c_k cos(2 pi j k / N) summed over all k (O(N^2))."""
    c = dif.window_column(N, L)
    j = np.arange(N)[:, None]
    k = np.arange(N)[None, :]
    lam = (c[None, :] * np.cos(2 * np.pi * j * k / N)).sum(1)
    assert np.max(np.abs(lam - closed_form_lambda(N, L))) < 1e-14


@pytest.mark.parametrize("N,L", [(12, 3), (12, 4), (64, 16), (60, 7), (4096, 512)])
def test_spectrum_invariants(N, L):
    lam = fif_spectral.eigenvalues(N, L)
    assert abs(lam[0] - 1.0) < 1e-15
    assert lam.min() > -1e-15 and lam.max() < 1 + 1e-15
    # only lambda_0 equals one (Theorem 4)
    assert np.all(lam[1:] < 1.0 - 1e-12)
    # exact zeros where L*j = 0 mod N, j != 0 (the kernel of W)
    zeros = [j for j in range(1, N) if (L * j) % N == 0]
    for j in zeros:
        assert abs(lam[j]) < 1e-15


# ------------------------------------------------------ one application ---

def dense_W(N: int, L: int) -> np.ndarray:
    """Dense circulant from the window definition, built independently:
    triangle h_q = (L-|q|)/L^2, w = h conv h, W_ij = sum over periodic images."""
    q = np.arange(-(L - 1), L)
    h = (L - np.abs(q)) / float(L * L)
    w = np.convolve(h, h)
    off = np.arange(-(2 * L - 2), 2 * L - 1)
    W = np.zeros((N, N))
    for i in range(N):
        for wq, d in zip(w, off):
            W[i, (i - d) % N] += wq
    return W


@pytest.mark.parametrize("N,L", [(3, 1), (5, 2), (8, 3), (13, 5), (16, 16), (20, 33), (64, 9)])
@pytest.mark.parametrize("form", [0, 1])
def test_apply_matches_dense_brute_force(N, L, form):
    rng = np.random.default_rng(N * 100 + L)
    x = rng.standard_normal(N)
    W = dense_W(N, L)
    assert np.max(np.abs(W @ x - dif.apply_window(x, L, form))) < 1e-14
    ev = np.linalg.eigvalsh(W)
    assert ev.min() > -1e-13 and abs(ev.max() - 1.0) < 1e-13
    # Theorem 4: W = I when L = 1 (c_0 = 1); otherwise lambda_0 = 1 is the only unit eigenvalue
    assert np.sum(ev > 1 - 1e-9) == (N if L == 1 else 1)


@pytest.mark.parametrize("N,L", [(31, 40), (257, 17), (1000, 77), (4096, 21), (4096, 4096),
                                 (4095, 999), (6000, 9000)])
def test_box_form_equals_literal(N, L):
    rng = np.random.default_rng(7 + N + L)
    x = rng.standard_normal(N)
    a0 = dif.apply_window(x, L, 0)
    a1 = dif.apply_window(x, L, 1)
    assert np.max(np.abs(a0 - a1)) < 1e-13 * np.max(np.abs(x))


@pytest.mark.parametrize("N,L,k0", [(64, 5, 3), (64, 5, 7), (128, 9, 20), (100, 13, 11), (4096, 21, 200)])
def test_pure_tone_decays_by_one_minus_lambda(N, L, k0):
    """A DFT mode is an eigenvector of the circulant: each step multiplies it
    by exactly 1 - lambda_{k0} and SD_m equals lambda_{k0} for every m."""
    i = np.arange(N)
    s = np.cos(2 * np.pi * k0 * i / N + 0.3)
    lam = closed_form_lambda(N, L)[k0]
    for form in (0, 1):
        x, sd, _ = dif.inner_trace(s, L, 5, form)
        assert np.max(np.abs(x - (1 - lam) ** 5 * s)) < 1e-13
        assert np.max(np.abs(sd - lam)) < 1e-13


# ---------------------------------------------------------------- extrema ---

def naive_extrema(v) -> int:
    """Collapse runs of equal values, then count strict interior extrema."""
    c = [v[0]]
    for x in v[1:]:
        if x != c[-1]:
            c.append(x)
    n = 0
    for a, b, d in zip(c, c[1:], c[2:]):
        if (b > a and b > d) or (b < a and b < d):
            n += 1
    return n


def test_extrema_exhaustive_small_patterns():
    for n in range(1, 9):
        for v in itertools.product((0.0, 1.0, 2.0), repeat=n):
            assert dif.count_extrema(np.array(v))[0] == naive_extrema(v), v


def test_extrema_plateaus_and_endpoints():
    assert dif.count_extrema([0, 1, 1, 1, 0])[0] == 1
    assert dif.count_extrema([0, 1, 1, 2, 3])[0] == 0
    assert dif.count_extrema([5, 0, 5])[0] == 1
    assert dif.count_extrema([1, 2, 3, 4])[0] == 0
    assert dif.count_extrema([3.0])[0] == 0
    N = 1000
    s = np.cos(2 * np.pi * 5 * np.arange(N) / N + 0.1)
    assert dif.count_extrema(s)[0] == 10


# ------------------------------------------------------ inner-loop laws ---

def test_sd_is_non_increasing():
    s = siggen.tones3()
    for L in (21, 104, 512):
        _, sd, _ = dif.inner_trace(s, L, 60, 1)
        assert np.all(np.diff(sd) <= 1e-13 * sd[:-1])


def test_theorem5_a_priori_bound():
    """For m >= N0 of the a-priori inequality, ||s_{m+1} - s_m|| < delta."""
    N, L = 128, 6
    s = siggen.tones3(N=N, freqs=(3.0, 11.0, 30.0))
    lam = closed_form_lambda(N, L)
    n_zero = int(np.sum(np.abs(lam) < 1e-15))
    st = np.fft.fft(s) / math.sqrt(N)  # unitary DFT: s~ = U^T s
    rhs_scale = np.max(np.abs(st)) * math.sqrt(N - 1 - n_zero)
    for delta in (1.0, 1e-1, 1e-2):
        # smallest n0 with n0^n0 / (n0+1)^(n0+1) < delta / rhs_scale, in logs
        n0 = 1
        while n0 * math.log(n0) - (n0 + 1) * math.log(n0 + 1) >= math.log(delta / rhs_scale):
            n0 += 1
        _, _, step = dif.inner_trace(s, L, n0 + 40, 1)
        # step[m] = ||s_{m+1} - s_m||, m = 0-based application count
        assert np.all(step[n0:] < delta)


# ------------------------------------------------- exact rational brute ---

def _exact_dif(s_int, delta: Fraction, max_imfs: int, max_inner: int = 400):
    """Algorithm 2 in exact rationals; same readings as the oracle."""
    N = len(s_int)
    r = [Fraction(int(v)) for v in s_int]
    out = []
    maxs = max(abs(v) for v in r)
    for _ in range(max_imfs):
        mean = sum(r) / N
        if max(abs(v - mean) for v in r) <= Fraction(1, 10**9) * maxs:
            break
        k = naive_extrema(r)
        if k < 2:
            break
        L = -(-2 * N // k)
        q = range(-(L - 1), L)
        h = {d: Fraction(L - abs(d), L * L) for d in q}
        w = {}
        for a in q:
            for b in q:
                w[a + b] = w.get(a + b, 0) + h[a] * h[b]
        c = [Fraction(0)] * N
        for d, v in w.items():
            c[d % N] += v
        x = list(r)
        m = 0
        while True:
            a = [sum(c[p] * x[(i - p) % N] for p in range(N)) for i in range(N)]
            na = sum(v * v for v in a)
            nx = sum(v * v for v in x)
            x = [xi - ai for xi, ai in zip(x, a)]
            m += 1
            if nx == 0 or na <= delta * delta * nx:
                break
            if m >= max_inner:
                return None
        out.append((k, L, m, x))
        r = [ri - xi for ri, xi in zip(r, x)]
    return out, r


@pytest.mark.parametrize("seed", range(6))
def test_exact_rational_decisions(seed):
    rng = np.random.default_rng(1000 + seed)
    N = int(rng.integers(8, 15))
    s = rng.integers(-20, 21, size=N)
    delta = Fraction(1, 10)
    ex = _exact_dif(list(s), delta, 3)
    if ex is None:
        pytest.skip("exact iteration exceeded its cap")
    steps, rem = ex
    d = dif.decompose(s.astype(float), 0.1, 3, inner_form=0)
    assert [t[0] for t in steps] == d.k
    assert [t[1] for t in steps] == d.L
    assert [t[2] for t in steps] == d.m
    for (k, L, m, x), imf in zip(steps, d.imfs):
        assert np.max(np.abs(np.array([float(v) for v in x]) - imf)) < 1e-12
    assert np.max(np.abs(np.array([float(v) for v in rem]) - d.remainder)) < 1e-12


# ------------------------------------------------------ whole-method laws ---

@pytest.fixture(scope="module")
def tones_dec():
    """The three-tone signal decomposed by the literal iteration (folded
    taps, one tap sum per output sample; about 4 s)."""
    s = siggen.tones3()
    return s, dif.decompose(s, 1e-3, 8, inner_form=0)


def test_reconstruction_and_zero_mean(tones_dec):
    s, d = tones_dec
    assert np.max(np.abs(d.imfs.sum(0) + d.remainder - s)) < 1e-13 * np.max(np.abs(s))
    for imf in d.imfs:
        assert abs(imf.mean()) < 1e-15 * np.max(np.abs(s))
    assert abs(d.remainder.mean() - s.mean()) < 1e-15


def test_three_tones_separate(tones_dec):
    """The mask-length reading makes the first three IMFs the 200, 40 and 8
    cycle components (a semantic check of the window-length reading)."""
    s, d = tones_dec
    x = siggen.grid(s.size)
    comps = [(1 + 0.3 * sg * np.sin(2 * np.pi * x)) * np.cos(2 * np.pi * f * x)
             for f, sg in ((200, 1), (40, -1), (8, 1))]
    for imf, c in zip(d.imfs[:3], comps):
        assert np.corrcoef(imf, c)[0, 1] > 0.999
    # a residual led by a tone of f cycles has about 2f extrema (one maximum
    # and one minimum per cycle); the mask length then follows its rule
    for kj, Lj, f in zip(d.k[:3], d.L[:3], (200, 40, 8)):
        assert abs(kj - 2 * f) <= 2, (kj, f)
        assert Lj == -(-2 * s.size // kj)
    assert all(sd <= 1e-3 for sd in d.sd)
    assert all(p > 1e-3 for p in d.sd_prev)


def test_literal_and_box_oracles_agree(tones_dec):
    """The literal folded-tap iteration and the four-box-sum form of W give
    the same decomposition of the three-tone signal (N = 4096)."""
    s, d = tones_dec
    e = dif.decompose(s, 1e-3, 8, inner_form=1)
    assert d.n_imfs == e.n_imfs >= 4
    assert (d.k, d.L, d.m) == (e.k, e.L, e.m)
    scale = np.linalg.norm(s)
    for a, b in zip(d.imfs, e.imfs):
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a) + 1e-15 * scale


def _assert_same_decomposition(d, e, s):
    assert (d.k, d.L, d.m) == (e.k, e.L, e.m)
    scale = np.linalg.norm(s)
    for a, b in zip(d.imfs, e.imfs):
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a) + 1e-15 * scale
    assert np.linalg.norm(d.remainder - e.remainder) <= 1e-12 * scale


def test_direct_form_equals_iteration_tones(tones_dec):
    """Theorem 5: the one-step spectral form reproduces the iteration."""
    s, d = tones_dec
    _assert_same_decomposition(d, fif_spectral.decompose(s, 1e-3, 8), s)


@pytest.mark.parametrize("N", [96, 350, 1001, 2048])
def test_direct_form_equals_iteration_random(N):
    s = siggen.tones3(N=N, freqs=(N / 40, N / 9, N / 3.3), seed_index=N)
    _assert_same_decomposition(dif.decompose(s, 1e-3, 6), fif_spectral.decompose(s, 1e-3, 6), s)


@pytest.mark.slow
def test_direct_form_equals_iteration_chirps():
    s = siggen.chirps(3)
    d = dif.decompose(s, 1e-3, 12)
    _assert_same_decomposition(d, fif_spectral.decompose(s, 1e-3, 12), s)


def test_equivariances():
    s = siggen.tones3(N=1024, freqs=(5, 23, 101), seed_index=4)
    d = dif.decompose(s, 1e-3, 6, inner_form=1)
    for t, inv in ((lambda v: 4.0 * v, lambda v: v / 4.0), (lambda v: -v, lambda v: -v)):
        e = dif.decompose(t(s), 1e-3, 6, inner_form=1)
        assert (d.k, d.L, d.m) == (e.k, e.L, e.m)
        assert np.array_equal(d.imfs, inv(e.imfs))
    e = dif.decompose(s[::-1].copy(), 1e-3, 6, inner_form=1)
    assert (d.k, d.L, d.m) == (e.k, e.L, e.m)
    assert np.max(np.abs(d.imfs - e.imfs[:, ::-1])) < 1e-12


def test_decomposition_is_not_linear():
    """Section 2: the filter length depends on the signal, so IMFs(p+q) is
    not IMFs(p) + IMFs(q) in general."""
    N = 1024
    x = siggen.grid(N)
    p = np.cos(2 * np.pi * 50 * x)
    q = 0.7 * np.cos(2 * np.pi * 7 * x + 0.4)
    dp, dq, dpq = (dif.decompose(v, 1e-3, 3, inner_form=1) for v in (p, q, p + q))
    assert dp.L[0] != dpq.L[0] or dq.L[0] != dpq.L[0]
    assert np.max(np.abs(dpq.imfs[0] - dp.imfs[0] - dq.imfs[0])) > 1e-3


def test_cap_on_a_pure_tone():
    """A single DFT mode never satisfies SD <= delta when lambda > delta; the
    cap ends the inner loop with m = max_inner and the cap flag."""
    N = 256
    s = np.cos(2 * np.pi * 8 * np.arange(N) / N)
    d = dif.decompose(s, 1e-6, 1, max_inner=50, inner_form=1)
    assert d.m == [50] and d.flags == [dif.FLAG_CAP]
    lam = closed_form_lambda(N, d.L[0])[8]
    assert abs(d.sd[0] - lam) < 1e-13


def test_stop_rules():
    d = dif.decompose(np.full(64, 3.25), 1e-3, 5)
    assert d.n_imfs == 0 and d.stop_reason == dif.STOP_FLOOR
    d = dif.decompose(np.zeros(64), 1e-3, 5)
    assert d.n_imfs == 0 and d.stop_reason == dif.STOP_FLOOR
    d = dif.decompose(np.linspace(0, 1, 64) ** 2, 1e-3, 5)
    assert d.n_imfs == 0 and d.stop_reason == dif.STOP_FEW_EXTREMA
    s = siggen.tones3(N=512, freqs=(3, 17, 60))
    d = dif.decompose(s, 1e-3, 2)
    assert d.n_imfs == 2 and d.stop_reason == dif.STOP_MAX_IMFS


def test_mask_rules():
    assert dif.mask_length(4096, 401, 0) == 21
    assert dif.mask_length(4096, 2, 0) == 4096
    assert dif.mask_length(10, 3, 0) == 7
    assert dif.mask_length(4096, 401, 1, 1.6) == 2 * math.floor(1.6 * 4096 / 401)
    assert dif.mask_length(100, 7, 1, 1.6) == 44


def test_degenerate_tail_time_domain_stops_at_the_rounding_level():
    """A pure tone whose eigenvalue exceeds delta: in exact arithmetic every
    iterate is the tone times (1 - lambda)^m, so SD_m = lambda > delta for
    every m and the inner loop can only end at the cap (equation "SD", the
    cap stated beside it).  The FP64 time-domain iteration keeps SD = lambda
    while the tone is representable, then stops once the tone has decayed to
    the rounding level of the signal, at a step count that depends on the
    order of the roundings (literal taps and box sums differ).  The direct
    form with the noise-floor reading returns the cap, the exact-arithmetic
    answer; that reading decides on such tails."""
    N, k0, delta = 256, 8, 5e-4
    s = np.cos(2 * np.pi * k0 * np.arange(N) / N + 0.3)
    lit = dif.decompose(s, delta, 1, mask_rule=1, inner_form=0)
    box = dif.decompose(s, delta, 1, mask_rule=1, inner_form=1)
    spec = fif_spectral.decompose(s, delta, 1, mask_rule=1)
    assert lit.L == box.L == spec.L
    lam = closed_form_lambda(N, lit.L[0])[k0]
    assert lam > delta
    # exact answer: the cap, SD = lambda
    assert spec.m == [1_000_000] and spec.flags == [dif.FLAG_CAP]
    assert abs(spec.sd[0] - lam) <= 1e-15
    # time domain: SD = lambda to rounding for the first 2000 steps ...
    _, sd, _ = dif.inner_trace(s, lit.L[0], 2000, form=1)
    assert np.max(np.abs(sd - lam)) < 1e-15
    # ... and its stop comes only where the exact iterate (1 - lambda)^m has
    # fallen below 1e-15 of the tone, at a rounding-dependent m
    for d in (lit, box):
        assert d.m[0] < 1_000_000 and d.flags == [0]
        assert (1.0 - lam) ** d.m[0] < 1e-15
        assert (1.0 - lam) ** (d.m[0] - 2000) > 1e-15
    assert lit.m != box.m


def test_imfs_at_given_decisions_repeat_the_decomposition():
    """fif_spectral.imfs_at with the (L, m) the direct form chose gives its
    IMFs and remainder (the same formula on the half spectrum: equal up to
    FFT rounding)."""
    s = siggen.tones3(N=2048, freqs=(6, 31, 150), seed_index=9)
    d = fif_spectral.decompose(s, 1e-3, 6)
    imfs, rem = fif_spectral.imfs_at(s, d.L, d.m)
    sn = np.linalg.norm(s)
    assert imfs.shape == d.imfs.shape
    for a, b in zip(imfs, d.imfs):
        assert np.linalg.norm(a - b) <= 1e-14 * sn
    assert np.linalg.norm(rem - d.remainder) <= 1e-14 * sn
