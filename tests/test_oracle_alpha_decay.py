"""Pins of the alpha_t schedule of exact mode (alpha_decay): alpha shrinks
with the bin count, each round's window grows with 1 / alpha_r and still
meets the flat-window accuracy, and planted spectra are recovered exactly."""
import numpy as np
import pytest

import siggen
from oracle.exact import noiseless_sparse_fft
from oracle.fft import fft_radix2
from oracle.params import SfftParams
from oracle.window import default_w, gprime, window_time


def params(n, k, B, b_min, alpha_decay, rounds=10, seed=1, delta=1e-9):
    return SfftParams(n=n, k=k, B=B, w=default_w(n, B, 0.5, delta), seed=seed, alpha=0.5, delta=delta,
                      theta=0.05, g_min=0.25, rounds=rounds, b_min=b_min, patience=4, alpha_decay=alpha_decay)


def test_schedule_halves_alpha_with_B_then_holds():
    p = params(1 << 16, 8, 1024, 64, 0.5)
    Bs = [p.round_bins(r)[0] for r in range(10)]
    assert Bs == [1024, 512, 256, 128, 64, 64, 64, 64, 64, 64]
    alphas = [p.round_alpha(r) for r in range(10)]
    assert alphas == [0.5, 0.25, 0.125, 0.0625] + [0.03125] * 6
    # sigma_g scales as B_r / alpha_r, and so does w_r: B_r halves and alpha_r halves, w_r stays
    w0 = p.round_bins(0)[1]
    assert all(p.round_bins(r)[1] == w0 for r in range(10))
    assert w0 == p.w


@pytest.mark.parametrize("decay", [0.0, 1.0])
def test_no_decay_is_the_fixed_schedule(decay):
    p = params(1 << 16, 8, 1024, 64, decay)
    q = params(1 << 16, 8, 1024, 64, 0.0)
    for r in range(10):
        assert p.round_alpha(r) == 0.5
        assert p.round_bins(r) == (q.B >> min(r, 4), q.w * (q.B >> min(r, 4)) // q.B)


def test_decay_rounds_up_to_a_multiple_of_B_r():
    p = params(1 << 16, 8, 1024, 64, 0.7)
    for r in range(10):
        Br, wr = p.round_bins(r)
        f = 0.7 ** min(r, 4)
        assert wr % Br == 0 and wr >= p.w // p.B * Br / f - 1e-6 and wr < (p.w // p.B / f + 1) * Br


def test_decayed_windows_meet_the_flat_window_accuracy():
    """||Ghat_r - G'_r||_inf < delta for every round of the schedule (flat
    window definition, fourth bullet): a window that kept the fixed-alpha
    length w B_r / B would fall short as alpha_r shrinks."""
    n, delta = 1 << 14, 1e-9
    p = params(n, 8, 64, 16, 0.5, rounds=3, delta=delta)
    f = np.arange(n)
    fs = np.where(f >= n // 2, f - n, f)
    for r in range(3):
        Br, wr = p.round_bins(r)
        ar = p.round_alpha(r)
        assert wr < n
        G = window_time(n, Br, wr, ar, delta)
        g = np.zeros(n)
        t = np.arange(-(wr // 2), wr - wr // 2)
        g[t % n] = G
        Gh = fft_radix2(g)
        Gp = np.array([gprime(v, n, Br, ar, delta) for v in fs])
        assert np.max(np.abs(Gh - Gp)) < delta, r
        # the flat band widens as alpha_r shrinks: (1 - alpha_r) n / (2 B_r)
        assert gprime(int((1 - ar) * n / (2 * Br)), n, Br, ar, delta) == 1.0
    # the fixed-alpha window length is too short for the last round's alpha
    Br, wr = p.round_bins(2)
    short = p.w * Br // p.B
    assert short < wr
    G = window_time(n, Br, short, p.round_alpha(2), delta)
    g = np.zeros(n)
    t = np.arange(-(short // 2), short - short // 2)
    g[t % n] = G
    Gp = np.array([gprime(v, n, Br, p.round_alpha(2), delta) for v in fs])
    assert np.max(np.abs(fft_radix2(g) - Gp)) > delta


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_planted_spectra_recovered_exactly_with_decay(seed):
    n, k = 1 << 14, 12
    x, sup, val = siggen.planted_signal(n, k, 900 + seed, np.complex128, magnitude="unit")
    p = params(n, k, 64, 16, 0.5, rounds=16, seed=seed)
    res = noiseless_sparse_fft(x, p)
    assert np.array_equal(res.indices, np.sort(sup))
    order = np.argsort(sup)
    assert np.max(np.abs(res.values - val[order])) < 1e-9
