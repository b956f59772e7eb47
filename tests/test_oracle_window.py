"""Pins of the flat window (Section 2 definition, Section 7 construction)."""
import math

import numpy as np
import pytest

from oracle.fft import fft_radix2
from oracle.window import default_w, g_star, gprime, phi, window_shape, window_time


def dft_of_window(n, B, w, alpha, delta):
    G = window_time(n, B, w, alpha, delta)
    g = np.zeros(n)
    t = np.arange(-(w // 2), w - w // 2)
    g[t % n] = G
    return fft_radix2(g)          # sum_t G_t omega^{f t}: the bins' response at offset -f


@pytest.mark.parametrize("n,B,alpha,delta", [(8192, 64, 0.5, 1e-9), (16384, 64, 0.5, 1e-12),
                                             (16384, 64, 0.25, 1e-6), (8192, 32, 0.5, 1e-12)])
def test_window_spectrum_within_delta_of_gprime(n, B, alpha, delta):
    """||Ghat - G'||_inf < delta (flat window definition, fourth bullet)."""
    w = default_w(n, B, alpha, delta)
    assert w < n
    Gh = dft_of_window(n, B, w, alpha, delta)
    f = np.arange(n)
    fs = np.where(f >= n // 2, f - n, f)
    Gp = np.array([gprime(v, n, B, alpha, delta) for v in fs])
    assert np.max(np.abs(Gh.imag)) < delta          # G is real and even up to one edge sample
    assert np.max(np.abs(Gh - Gp)) < delta


def test_gprime_flat_and_stop_bands():
    n, B, alpha, delta = 1 << 14, 64, 0.5, 1e-9
    f = np.arange(-n // 2, n // 2)
    g = np.array([gprime(v, n, B, alpha, delta) for v in f])
    assert np.all((g >= 0.0) & (g <= 1.0))
    assert np.all(g[np.abs(f) <= (1 - alpha) * n / (2 * B)] == 1.0)
    assert np.all(g[np.abs(f) >= n / (2 * B)] == 0.0)
    # symmetric and monotone in |f|
    assert np.array_equal(g, np.array([gprime(-v, n, B, alpha, delta) for v in f]))
    pos = g[n // 2:]
    assert np.all(np.diff(pos) <= 0.0)


def test_phi_properties_and_marsaglia_series():
    """The CDF claim of Section 7: symmetry, the tail bound, and the Taylor
    series Phi(t) = 1/2 + pdf(t) (t + t^3/3 + t^5/(3*5) + ...)."""
    for t in np.linspace(-6, 6, 49):
        assert abs(phi(t) - (1 - phi(-t))) < 1e-15
        if t < 0:
            assert phi(t) <= math.exp(-t * t / 2)
        term, s, j = t, 0.0, 1
        while abs(term) > 1e-300 and j < 400:
            s += term
            term *= t * t / (2 * j + 1)
            j += 1
        series = 0.5 + math.exp(-t * t / 2) / math.sqrt(2 * math.pi) * s
        assert abs(series - phi(t)) < 1e-13


def test_gstar_centre_and_continuity():
    sg, C = window_shape(1 << 14, 64, 0.5, 1e-9)
    assert g_star(0, sg, C) == 2 * C
    assert abs(g_star(1e-7, sg, C) - 2 * C) < 1e-10


def test_window_length_is_order_B_over_alpha_log():
    """|supp G| = O((B / alpha) log(n / delta))."""
    for (n, B, alpha, delta) in [(1 << 14, 64, 0.5, 1e-12), (1 << 20, 1024, 0.5, 1e-6), (1 << 22, 1024, 0.5, 1e-9)]:
        w = default_w(n, B, alpha, delta)
        ratio = w / ((B / alpha) * math.log(n / delta))
        assert 0.5 < ratio < 4.0
        assert w % B == 0
