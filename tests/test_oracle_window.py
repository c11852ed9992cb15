"""Pins of the spectral oracle's sampled window shapes (Section 4: the
direct method needs only the DFT of W's first column, equation "Lambdas",
which can be tabulated for any filter).

Each construction step is pinned to something outside it: hand-computed
taps, the closed forms of the triangle (equation "eig2") and of the box
(a Dirichlet kernel), the C time-domain oracle's window column, and a literal
time-domain iteration written out here with explicit loops.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import siggen
from oracle import dif
from oracle import fif_spectral as fs


def test_shape_taps_by_hand():
    # flat top then a linear edge, K = 2, L = 4: x = |q|/4 -> 1, 1, 1, 0.5
    h = fs.shape_taps(4, [1.0, 1.0, 0.0])
    assert np.array_equal(h, [0.5, 1.0, 1.0, 1.0, 1.0, 1.0, 0.5])
    # the triangle: (L - |q|) / L
    assert np.allclose(fs.shape_taps(5, [1.0, 0.0]) * 5, [1, 2, 3, 4, 5, 4, 3, 2, 1], rtol=0, atol=1e-15)
    # K = 3, L = 2: x = 0, 1/2 -> samples 0 and 1.5 (between i = 1 and 2)
    assert np.allclose(fs.shape_taps(2, [4.0, 2.0, 1.0, 0.0]), [1.5, 4.0, 1.5], rtol=0, atol=1e-15)


@pytest.mark.parametrize("N,L", [(64, 3), (128, 6), (1000, 17), (4096, 21), (97, 60), (64, 64)])
def test_triangle_shape_is_the_default_window(N, L):
    c = fs.window_column_shape(N, L, [1.0, 0.0])
    assert np.max(np.abs(c - dif.window_column(N, L))) <= 1e-15
    lam = fs.eigenvalues_shape(N, L, [1.0, 0.0])
    assert np.max(np.abs(lam - fs.eigenvalues_closed(N, L))) <= 1e-14


@pytest.mark.parametrize("N,L", [(64, 3), (128, 10), (1000, 17), (4096, 300)])
def test_box_shape_is_a_squared_dirichlet_kernel(N, L):
    """Shape [1, 1]: h is a box of 2L-1 taps, lambda_j = [sin(pi M j/N) /
    (M sin(pi j/N))]^2 with M = 2L - 1 (for 4L-3 <= N: no folding)."""
    M = 2 * L - 1
    j = np.arange(1, N, dtype=np.int64)
    # |sin(pi M j / N)| with M j reduced modulo N exactly (the square hides the sign)
    t = (M * j) % N
    t = np.minimum(t, N - t)
    u = np.minimum(j, N - j)
    d = np.sin(np.pi * t / N) / (M * np.sin(np.pi * u / N))
    lam = fs.eigenvalues_shape(N, L, [1.0, 1.0])
    assert lam[0] == 1.0
    assert np.max(np.abs(lam[1:] - d * d)) <= 1e-14


@pytest.mark.parametrize("N,L,K", [(128, 9, 5), (1000, 40, 17), (256, 200, 3), (97, 12, 64), (64, 50, 2)])
def test_shape_eigenvalues_are_the_dft_of_the_column(N, L, K):
    """(DFT h)^2 / (sum h)^2 = DFT of the folded h * h / (sum h)^2 (the
    convolution theorem), up to rounding and the exact-zero reading."""
    shape = np.random.default_rng(N + L).uniform(0.05, 1.0, K + 1)
    a = fs.eigenvalues_shape(N, L, shape)
    b = np.fft.fft(fs.window_column_shape(N, L, shape)).real
    assert np.max(np.abs(a - b)) <= 1e-15


def test_exact_zeros_of_a_box_spectrum():
    """Shape [1, 1] at L = 2 is the box [1, 1, 1]: H_j = (1 + 2 cos(2 pi j/N))/3
    vanishes at j = N/3 and 2N/3; those eigenvalues are exactly 0."""
    lam = fs.eigenvalues_shape(30, 2, [1.0, 1.0])
    assert lam[10] == 0.0 and lam[20] == 0.0
    assert np.count_nonzero(lam == 0.0) == 2


def test_shape_eigenvalues_lie_in_the_unit_interval():
    rng = np.random.default_rng(3)
    for N, L, K in ((128, 9, 5), (1000, 40, 17), (256, 200, 3), (97, 12, 64)):
        shape = rng.uniform(0.0, 1.0, K + 1)
        lam = fs.eigenvalues_shape(N, L, shape)
        assert lam[0] == 1.0
        assert np.all(lam >= -1e-15) and np.all(lam <= 1.0 + 1e-15)
        assert np.max(np.abs(lam[1:] - lam[1:][::-1])) <= 1e-15


def _literal_decompose_one(s, L, h, delta, max_inner=100000):
    """One IMF by the time-domain iteration of Algorithm 2 with the window
    h * h / (sum h)^2 applied literally (two circular convolutions by h)."""
    N = s.size
    R = (len(h) - 1) // 2
    S = sum(h)

    def conv(x):
        y = np.zeros(N)
        for i in range(N):
            acc = 0.0
            for t in range(-R, R + 1):
                acc += h[t + R] * x[(i - t) % N]
            y[i] = acc
        return y

    x = s.copy()
    m = 0
    while True:
        a = conv(conv(x)) / (S * S)
        sd = math.sqrt(float(np.dot(a, a)) / float(np.dot(x, x)))
        x = x - a
        m += 1
        if sd <= delta or m >= max_inner:
            return x, m, sd


@pytest.mark.parametrize("shape,N", [([1.0, 1.0, 0.0], 96), ([1.0, 0.7, 0.2, 0.0], 128),
                                     ([0.5, 1.0, 0.25], 80)])
def test_shape_decomposition_matches_the_literal_iteration(shape, N):
    """Theorem 5 for a general symmetric window: the first IMF of the
    spectral oracle equals the literal time-domain iteration (same m)."""
    s = siggen.tones3(N=N, freqs=(2.0, 7.0, 19.0))
    delta = 1e-2
    d = fs.decompose(s, delta, 1, window=shape)
    L = d.L[0]
    h = list(fs.shape_taps(L, shape))
    imf, m, sd = _literal_decompose_one(s, L, h, delta)
    assert d.m[0] == m
    assert d.sd[0] == pytest.approx(sd, rel=1e-9)
    assert np.max(np.abs(d.imfs[0] - imf)) <= 1e-12 * np.max(np.abs(s))


def test_triangle_shape_decomposes_like_the_default():
    s = siggen.chirps(2, N=8192)
    a = fs.decompose(s, 1e-3, 6)
    b = fs.decompose(s, 1e-3, 6, window=[1.0, 0.0])
    assert (a.k, a.L, a.m) == (b.k, b.L, b.m)
    assert np.max(np.abs(a.imfs - b.imfs)) <= 1e-12 * np.max(np.abs(s))


def test_shape_with_the_apriori_count_is_refused():
    with pytest.raises(ValueError):
        fs.decompose(siggen.tones3(N=256), 1e-3, 1, stop="apriori", window=[1.0, 0.0])
