"""Pins of the spectral oracle's variants: the absolute stop criterion, the
a-priori N0 of Theorem 5, the thresholded IMF and the spectral-peak mask
length.  Each is checked against the time-domain iteration, a closed form
on pure tones, or a bound the paper proves.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import siggen
from oracle import dif
from oracle import fif_spectral as fs


def _tone(N, k0, amp=1.0, phase=0.3):
    i = np.arange(N)
    return amp * np.cos(2 * np.pi * k0 * i / N + phase)


# ----------------------------------------------- closed-form eigenvalues --

@pytest.mark.parametrize("N,L", [(64, 3), (128, 6), (1000, 17), (4096, 21), (4096, 2048), (97, 200)])
def test_closed_form_eigenvalues_equal_the_column_dft(N, L):
    """eq. "eig2" against the DFT of the window column (eq. "Lambdas")."""
    a = fs.eigenvalues_closed(N, L)
    b = fs.eigenvalues(N, L)
    assert np.max(np.abs(a - b)) <= 1e-14
    assert a[0] == 1.0 and np.all(a >= 0.0) and np.all(a <= 1.0)


# ------------------------------------------------------ bisection search --

@pytest.mark.parametrize("delta", [1e-3, 1e-4])
def test_bisection_search_equals_linear_scan(delta):
    """SD_m is non-increasing, so bisection must find the linear scan's m."""
    for s in (siggen.tones3(), siggen.chirps(3, N=8192), siggen.uneven_signal(5, 6000)):
        a = fs.decompose(s, delta, 6)
        b = fs.decompose(s, delta, 6, search="bisect")
        assert (a.k, a.L, a.m) == (b.k, b.L, b.m)
        assert np.allclose(a.sd, b.sd, rtol=1e-9, atol=0)
        assert np.max(np.abs(a.imfs - b.imfs)) <= 1e-12 * np.max(np.abs(s))


# ------------------------------------------------------- absolute criterion --

@pytest.mark.parametrize("delta", [1e-1, 1e-2, 3e-3])
def test_absolute_stop_matches_time_domain_iteration(delta):
    """m = smallest m >= 1 with ||s_{m+1} - s_m||_2 < delta, the step norms
    taken from the literal time-domain iteration."""
    N = 256
    s = siggen.tones3(N=N, freqs=(3.0, 11.0, 40.0))
    d = fs.decompose(s, delta, 1, stop="abs")
    L = d.L[0]
    _, _, step = dif.inner_trace(s, L, 3000, 1)
    # step[m] = ||s_{m+1} - s_m||, m counted from 0
    m_td = next(m for m in range(1, step.size) if step[m] < delta)
    assert d.m[0] == m_td
    assert d.sd[0] == pytest.approx(step[m_td], rel=1e-10)
    assert d.sd_prev[0] == pytest.approx(step[m_td - 1], rel=1e-10)


def test_absolute_stop_on_a_pure_tone():
    """||W s_m|| = lambda (1 - lambda)^m ||s|| for an eigenvector."""
    N, k0 = 1024, 37
    s = _tone(N, k0)
    delta = 1e-2
    d = fs.decompose(s, delta, 1, stop="abs")
    L = d.L[0]
    lam = float(np.sin(np.pi * L * k0 / N) / (L * np.sin(np.pi * k0 / N))) ** 4
    ns = float(np.linalg.norm(s))
    m = 1
    while lam * (1 - lam) ** m * ns >= delta:
        m += 1
    assert d.m[0] == m


# ---------------------------------------------------------- a-priori N0 --

def test_zero_eigenvalue_count():
    for N, L in ((128, 6), (120, 40), (64, 64), (210, 35), (97, 5)):
        lam = fs.eigenvalues(N, L)
        assert fs.zero_eigenvalues(N, L) == math.gcd(L, N) - 1
        assert fs.zero_eigenvalues(N, L) == int(np.sum(np.abs(lam[1:]) < 1e-12))


@pytest.mark.parametrize("delta", [1.0, 0.3, 0.1])
def test_apriori_n0_satisfies_theorem5(delta):
    """Theorem 5: for m >= N0, ||s_{m+1} - s_m|| < delta; so the a-priori
    count is never below the absolute criterion's."""
    N = 128
    s = siggen.tones3(N=N, freqs=(3.0, 11.0, 30.0))
    d = fs.decompose(s, delta, 1, stop="apriori")
    n0, L = d.m[0], d.L[0]
    _, _, step = dif.inner_trace(s, L, n0 + 40, 1)
    assert np.all(step[n0:] < delta)
    da = fs.decompose(s, delta, 1, stop="abs")
    assert da.L[0] == L and da.m[0] <= n0


def test_apriori_n0_is_minimal():
    """N0 - 1 does not satisfy the inequality (evaluated here with exact
    rationals, independently of the oracle's logarithms)."""
    from fractions import Fraction
    N = 64
    s = siggen.tones3(N=N, freqs=(2.0, 5.0, 13.0))
    R = np.fft.fft(s)
    for L in (4, 7, 12):
        for delta in (2.0, 0.5):
            n0 = fs.apriori_n0(R, N, L, delta)
            rest = N - 1 - (math.gcd(L, N) - 1)
            bound = delta / (float(np.max(np.abs(R))) / math.sqrt(N) * math.sqrt(rest))
            b = Fraction(bound)

            def holds(n):
                return Fraction(n ** n, (n + 1) ** (n + 1)) < b
            assert holds(n0)
            assert n0 == 1 or not holds(n0 - 1)


# ------------------------------------------------------ thresholded IMF --

def test_threshold_vanishing_gamma_is_the_plain_imf():
    s = siggen.tones3()
    a = fs.decompose(s, 1e-3, 5)
    b = fs.decompose(s, 1e-3, 5, gamma=1e-300)
    assert (a.k, a.L, a.m) == (b.k, b.L, b.m)
    assert np.array_equal(a.imfs, b.imfs)


@pytest.mark.parametrize("gamma", [1e-1, 1e-2, 1e-3])
def test_threshold_bound(gamma):
    """Discrete form of the bound behind the thresholding proposition:
    the IMF changes only on thresholded bins, by a factor 1 - (1-lambda)^m
    <= gamma there, so ||IMF^SC - IMF^TH||_2 <= gamma ||r||_2."""
    s = siggen.tones3()
    a = fs.decompose(s, 1e-3, 1)
    b = fs.decompose(s, 1e-3, 1, gamma=gamma)
    assert (a.k, a.L, a.m) == (b.k, b.L, b.m)
    assert np.linalg.norm(a.imfs[0] - b.imfs[0]) <= gamma * np.linalg.norm(s) * (1 + 1e-12)


def test_threshold_takes_a_slowly_decaying_tone_whole():
    N, k0 = 1024, 3
    s = _tone(N, k0) + 1e-3 * _tone(N, 200)
    d = fs.decompose(s, 1e-3, 1, gamma=0.5)
    L, m = d.L[0], d.m[0]
    lam = float(np.sin(np.pi * L * k0 / N) / (L * np.sin(np.pi * k0 / N))) ** 4
    g = (1 - lam) ** m
    expected = 1.0 if g >= 0.5 else g
    # the IMF's component at k0 is the tone scaled by the (thresholded) factor
    comp = np.fft.fft(d.imfs[0])[k0] / np.fft.fft(_tone(N, k0))[k0]
    assert abs(comp - expected) < 1e-12


# ------------------------------------------------ spectral-peak mask rule --

@pytest.mark.parametrize("N,f", [(1024, 37), (4096, 200), (1000, 3)])
def test_peak_rule_on_a_pure_tone_equals_count_rule(N, f):
    s = _tone(N, f)
    a = fs.decompose(s, 1e-3, 1)
    b = fs.decompose(s, 1e-3, 1, mask_rule=2)
    assert b.L[0] == -(-N // f)
    # the count rule sees 2f or 2f - 1 extrema (endpoints are not extrema)
    assert a.L[0] in (-(-2 * N // (2 * f)), -(-2 * N // (2 * f - 1)))


def test_peak_rule_picks_the_highest_significant_peak():
    N = 2048
    for a2, rho, f_exp in ((0.5, 0.1, 300), (0.2, 0.1, 40), (0.2, 0.01, 300)):
        s = _tone(N, 40) + a2 * _tone(N, 300)
        R = np.fft.fft(s)
        assert fs.peak_frequency(R, rho) == f_exp
        d = fs.decompose(s, 1e-3, 1, mask_rule=2, peak_rho=rho)
        assert d.L[0] == -(-N // f_exp)


# ------------------------------------------- degenerate SD tails (cap) --

def _lam_tone(N, L, k0):
    return float(np.sin(np.pi * L * k0 / N) / (L * np.sin(np.pi * k0 / N))) ** 4


@pytest.mark.parametrize("search", ["linear", "bisect"])
def test_pure_tone_above_delta_runs_to_the_cap(search):
    """A pure DFT mode has SD_m = lambda_k0 for every m (an eigenvector of W),
    so with lambda_k0 > delta no m satisfies the test: m is the cap, SD stays
    lambda_k0.  The paper's mask rule puts lambda_k0 near 1.6e-3; the cap is
    past the step where the tone's weight mu^(m-1) underflows FP64."""
    N, k0, delta = 256, 8, 5e-4
    cap = 1_000_000 if search == "bisect" else 300_000
    s = _tone(N, k0)
    d = fs.decompose(s, delta, 1, mask_rule=1, max_inner=cap, search=search)
    lam = _lam_tone(N, d.L[0], k0)
    assert lam > delta
    assert 2 * (cap - 1) * math.log1p(-lam) < math.log(1e-308)
    assert d.m[0] == cap and d.flags[0] & 1
    assert d.sd[0] == pytest.approx(lam, rel=1e-12)


def test_pure_tone_below_delta_stops_at_once():
    N, k0 = 1024, 3
    s = _tone(N, k0)
    d = fs.decompose(s, 0.5, 1)
    assert _lam_tone(N, d.L[0], k0) <= 0.5 and d.m[0] == 1


def test_two_tones_cross_over_where_the_closed_form_says():
    """Tone k0 with lambda0 > delta plus a tone k1 of power ratio eps with
    lambda1 < delta: SD_m^2 = (lambda0^2 q + lambda1^2) / (q + 1), q =
    (P0/P1) (mu0/mu1)^(m-1), reaches delta^2 at a closed-form m; the weaker
    tone is counted (far above the noise floor)."""
    N, delta = 4096, 1e-3
    k0, k1, amp1 = 5, 23, 1e-9
    s = _tone(N, k0) + amp1 * _tone(N, k1, phase=1.1)
    d = fs.decompose(s, delta, 1, mask_rule=1, search="bisect")
    L = d.L[0]
    l0, l1 = _lam_tone(N, L, k0), _lam_tone(N, L, k1)
    assert l0 > delta > l1
    lp = 2.0 * math.log(1.0 / amp1)                       # log(P0 / P1)
    lr = 2.0 * (math.log1p(-l0) - math.log1p(-l1))        # log(mu0 / mu1) < 0
    m = 1
    while True:
        q = math.exp(lp + (m - 1) * lr)
        if (l0 * l0 * q + l1 * l1) / (q + 1.0) <= delta * delta:
            break
        m += 1
    assert m > 1000 and d.m[0] == m
    assert fs.decompose(s, delta, 1, mask_rule=1).m[0] == m     # linear scan alike


def test_noise_floor_and_rescaling_leave_ordinary_signals_alone():
    """On signals whose SD crosses delta long before any weight underflows,
    the noise floor and the rescaled sums give the plain N0 = 1, 2, ... scan
    of equation "SD" (written out here without either)."""
    for s in (siggen.tones3(N=2048), siggen.chirps(5, N=4096), siggen.uneven_signal(9, 3000)):
        d = fs.decompose(s, 1e-3, 1)
        N = s.size
        R = np.fft.fft(s)
        lam = fs.eigenvalues_closed(N, d.L[0])
        P = np.abs(R) ** 2
        x = P.copy()
        m = 0
        while True:
            m += 1
            sd = math.sqrt(float(np.sum(x * lam * lam)) / float(np.sum(x)))
            if sd <= 1e-3:
                break
            x = x * (1.0 - lam) ** 2
        assert d.m[0] == m
        assert d.sd[0] == pytest.approx(sd, rel=1e-9)
