"""Pins of the kind-1 flat window (oracle/window.py): the Kaiser-Bessel taper
of the ideal low-pass meets the Section 2 definition of a flat window, checked
against the window's transform computed independently (a full FFT of the
zero-padded window), and the method recovers planted spectra with it."""
import math

import numpy as np
import pytest
import scipy.special

import siggen
from oracle.exact import noiseless_sparse_fft
from oracle.general import sparse_fft
from oracle.params import SfftParams
from oracle.window import bessel_i0, default_w, gprime, kaiser_w, window_time


def test_bessel_i0_matches_the_library_routine():
    x = np.linspace(0.0, 40.0, 161)
    assert np.max(np.abs(bessel_i0(x) / scipy.special.i0(x) - 1.0)) < 1e-14


def full_response(n, B, w, alpha, delta):
    """Ghat_f for every integer f: FFT of the zero-padded kind-1 window."""
    G = window_time(n, B, w, alpha, delta, kind=1)
    x = np.zeros(n)
    t = np.arange(-(w // 2), w - w // 2)
    x[t % n] = G
    return np.fft.fft(x)


@pytest.mark.parametrize("n,B,alpha,delta,shrink", [
    (1 << 12, 16, 0.5, 1e-6, 1), (1 << 14, 64, 0.5, 1e-9, 1), (1 << 14, 64, 0.5, 1e-12, 1),
    (1 << 16, 256, 0.75, 1e-8, 1), (1 << 22, 1024, 0.75, 1e-8, 1), (1 << 22, 1024, 0.75, 1e-8, 16),
])
def test_kaiser_window_meets_the_flat_window_definition(n, B, alpha, delta, shrink):
    """||Ghat - G'||_inf < delta over every integer frequency: G' is 1 in the
    pass band, 0 in the stop band and the window's own (real) response in
    between; shrink > 1 checks a late round (B / shrink bins, w / shrink)."""
    w = kaiser_w(n, B, alpha, delta) // shrink
    B //= shrink
    Gh = full_response(n, B, w, alpha, delta)
    f = np.minimum(np.arange(n), n - np.arange(n))
    gp = np.where(f * 2 * B <= (1 - alpha) * n, 1.0, 0.0)
    trans = np.nonzero((f * 2 * B > (1 - alpha) * n) & (f * 2 * B < n))[0]
    pick = trans[np.linspace(0, len(trans) - 1, 64).astype(int)]
    for q in pick:
        gp[q] = gprime(int(q), n, B, alpha, delta, kind=1, w=w)
        # the transition value is the response itself (within FP64 rounding)
        assert abs(gp[q] - min(1.0, max(0.0, Gh[q].real))) < 1e-12
    outside = np.ones(n, bool)
    outside[trans] = False
    err = np.abs(Gh - gp)
    assert err[outside].max() < delta
    assert err[pick].max() < delta
    assert np.abs(Gh.imag).max() < delta


def test_kaiser_window_is_about_half_the_gaussian():
    n, B, alpha, delta = 1 << 22, 1024, 0.75, 1e-8
    assert kaiser_w(n, B, alpha, delta) <= 0.55 * default_w(n, B, alpha, delta)


@pytest.mark.parametrize("seed", range(4))
def test_planted_recovery_with_the_kaiser_window(seed):
    """Exact mode, C1 shape (n = 2^14, k = 16, B = 64, complex128): supports
    exact and values within 1e-9 of the planted spectrum."""
    n, k, B, delta = 1 << 14, 16, 64, 1e-12
    w = default_w(n, B, 0.5, delta, kind=1)
    x, sup, val = siggen.planted_signal(n, k, 700 + seed, np.complex128)
    r = noiseless_sparse_fft(x, SfftParams(n=n, k=k, B=B, w=w, seed=seed, delta=delta, window=1))
    assert np.array_equal(r.indices, sup)
    assert np.max(np.abs(r.values - val)) < 1e-9


def test_general_mode_with_the_kaiser_window():
    """General mode, n = 2^14, k = 8, 5 % noise: l2/l2 error at most 2 (the
    guarantee of Section 1) and every head coefficient located."""
    n, k, B = 1 << 14, 8, 64
    w = default_w(n, B, 0.5, 1e-6, kind=1)
    x, sup, val = siggen.planted_signal(n, k, 33, np.complex128, noise_ratio=0.05)
    p = SfftParams(n=n, k=k, B=B, w=w, seed=3, delta=1e-6, rounds=7, window=1)
    r = sparse_fft(x, p)
    assert set(sup.tolist()) <= set(r.indices.tolist())
    X = np.fft.fft(x) / math.sqrt(n)
    est = np.zeros(n, complex)
    est[r.indices] = r.values
    top = np.argsort(-np.abs(X))[:k]
    tail = np.delete(X, top)
    assert np.linalg.norm(X - est) <= 2.0 * np.linalg.norm(tail)
