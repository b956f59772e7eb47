"""Pins of the permutation, the fold and HashToBins (Section 2 permutation
claim; Section 3 HashToBins lemma and its proof's computation steps)."""
import numpy as np
import pytest

from oracle.fft import fft_radix2, naive_dft, unitary_dft
from oracle.hashing import (bin_offset, hash_to_bins, hash_to_bins_raw, omega_pow,
                            perm_position)
from oracle.window import default_w, gprime, window_time

import siggen


def explicit_permutation(x, sigma, a, b):
    """(P_{sigma,a,b} x)_t = x_{sigma (t - a)} omega^{sigma b t}, element by element."""
    n = len(x)
    out = np.zeros(n, complex)
    for t in range(n):
        out[t] = x[(sigma * (t - a)) % n] * np.exp(-2j * np.pi * ((sigma * b * t) % n) / n)
    return out


@pytest.mark.parametrize("seed", range(4))
def test_permutation_claim(seed):
    """(P x)^_{pi(i)} = xhat_i omega^{a sigma i} for every i."""
    n = 256
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    sigma = int(rng.integers(0, n // 2)) * 2 + 1
    a, b = int(rng.integers(0, n)), int(rng.integers(0, n))
    xhat = naive_dft(x) / np.sqrt(n)
    phat = naive_dft(explicit_permutation(x, sigma, a, b)) / np.sqrt(n)
    for i in range(n):
        lhs = phat[perm_position(i, sigma, b, n)]
        rhs = xhat[i] * omega_pow(a * sigma * i, n)
        assert abs(lhs - rhs) < 1e-11


def test_fold_identity():
    """FFT_B(v)_j = yhat_{j n / B} (unnormalised) for v_r = sum_l y_{r + l B}."""
    n, B = 1024, 32
    rng = np.random.default_rng(5)
    y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v = y.reshape(n // B, B).sum(axis=0)
    Y = naive_dft(y)
    assert np.max(np.abs(fft_radix2(v) - Y[:: n // B])) < 1e-10


def test_bin_offset_reconstructs_position():
    n, B = 1 << 12, 64
    rng = np.random.default_rng(11)
    for _ in range(2000):
        i, b = int(rng.integers(0, n)), int(rng.integers(0, n))
        sigma = int(rng.integers(0, n // 2)) * 2 + 1
        h, o = bin_offset(i, sigma, b, n, B)
        assert 0 <= h < B and -n // (2 * B) <= o < n // (2 * B)
        assert (h * (n // B) + o) % n == perm_position(i, sigma, b, n)


@pytest.mark.parametrize("a", [0, 1, 77])
def test_hashtobins_exact_identity_with_true_window(a):
    """u_j = sum_i Ghat(j n/B - pi(i)) xhat_i omega^{a sigma i} exactly (dense x),
    where Ghat is the unnormalised DFT of the truncated window: the identity
    in the HashToBins lemma's proof before G' replaces Ghat."""
    n, B = 2048, 32
    alpha, delta = 0.5, 1e-9
    w = 512
    rng = np.random.default_rng(a)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    sigma, b = 2 * int(rng.integers(0, n // 2)) + 1, int(rng.integers(0, n))
    G = window_time(n, B, w, alpha, delta)
    g = np.zeros(n)
    g[np.arange(-(w // 2), w - w // 2) % n] = G
    Ghat = naive_dft(g)
    xhat = naive_dft(x) / np.sqrt(n)
    u = hash_to_bins_raw(x, sigma, a, b, B, G)
    for j in range(B):
        s = 0.0
        for i in range(n):
            s += Ghat[(j * (n // B) - perm_position(i, sigma, b, n)) % n] * xhat[i] * omega_pow(a * sigma * i, n)
        assert abs(u[j] - s) < 1e-10 * np.linalg.norm(xhat, 1)


@pytest.mark.parametrize("seed", range(3))
def test_hashtobins_lemma_with_gprime(seed):
    """u_j = sum_{h(i)=j} xhat_i G'_{-o(i)} omega^{a sigma i} +- delta ||xhat||_1."""
    n, k, B, alpha, delta = 1 << 14, 12, 64, 0.5, 1e-12
    w = default_w(n, B, alpha, delta)
    x, sup, val = siggen.planted_signal(n, k, 40 + seed, np.complex128)
    rng = np.random.default_rng(seed)
    sigma, a, b = 2 * int(rng.integers(0, n // 2)) + 1, int(rng.integers(0, n)), int(rng.integers(0, n))
    u = hash_to_bins_raw(x, sigma, a, b, B, window_time(n, B, w, alpha, delta))
    expect = np.zeros(B, complex)
    for i, v in zip(sup, val):
        h, o = bin_offset(i, sigma, b, n, B)
        expect[h] += v * gprime(-o, n, B, alpha, delta) * omega_pow(a * sigma * int(i), n)
    assert np.max(np.abs(u - expect)) <= delta * np.sum(np.abs(val)) + 1e-13 * np.sqrt(n)


def test_subtracting_the_whole_spectrum_empties_the_bins():
    """HashToBins step 4 with zhat = xhat leaves only the delta-level residue."""
    n, k, B, alpha, delta = 1 << 15, 10, 64, 0.5, 1e-12
    w = default_w(n, B, alpha, delta)
    assert w < n
    x, sup, val = siggen.planted_signal(n, k, 9, np.complex128)
    G = window_time(n, B, w, alpha, delta)
    zhat = {int(i): complex(v) for i, v in zip(sup, val)}
    for (sigma, a, b) in [(3, 0, 5), (1001, 1, 77), (4095, 123, 4000)]:
        u = hash_to_bins(x, zhat, sigma, a, b, B, G, alpha, delta)
        assert np.max(np.abs(u)) <= delta * np.sum(np.abs(val)) + 1e-13 * np.sqrt(n)


def test_sign_of_modulation_matters():
    """A flipped modulation sign breaks the closed form (guards the b term)."""
    n, B, alpha, delta = 1 << 12, 32, 0.5, 1e-12
    w = default_w(n, B, alpha, delta)
    x, sup, val = siggen.planted_signal(n, 1, 3, np.complex128)
    G = window_time(n, B, w, alpha, delta)
    sigma, b = 77, 1234
    u = hash_to_bins_raw(x, sigma, 0, b, B, G)
    h, o = bin_offset(int(sup[0]), sigma, b, n, B)
    assert abs(u[h] - val[0] * gprime(-o, n, B, alpha, delta)) < 1e-10
    u_bad = hash_to_bins_raw(x, sigma, 0, (-b) % n, B, G)
    assert abs(u_bad[h] - val[0] * gprime(-o, n, B, alpha, delta)) > 1e-3
