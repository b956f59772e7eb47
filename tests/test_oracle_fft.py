"""Pins of the oracle's transforms (Section 2 convention) against the plain
definition and closed forms."""
import numpy as np
import pytest

from oracle.fft import fft_radix2, naive_dft, unitary_dft, unitary_idft


@pytest.mark.parametrize("n", [2, 4, 8, 64, 512, 4096])
def test_radix2_matches_naive_definition(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = naive_dft(x)
    got = fft_radix2(x)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.linalg.norm(ref)


def test_single_tone_is_one_spike():
    n, f0 = 1024, 337
    t = np.arange(n)
    x = np.exp(2j * np.pi * f0 * t / n)          # inverse-transform sign: spike at +f0
    X = unitary_dft(x)
    expect = np.zeros(n, complex)
    expect[f0] = np.sqrt(n)
    assert np.max(np.abs(X - expect)) < 1e-10


def test_boxcar_is_dirichlet_kernel():
    n, L = 2048, 37
    x = np.zeros(n, complex)
    x[:L] = 1.0
    X = fft_radix2(x)
    f = np.arange(1, n)
    dirichlet = np.exp(-1j * np.pi * f * (L - 1) / n) * np.sin(np.pi * f * L / n) / np.sin(np.pi * f / n)
    assert abs(X[0] - L) < 1e-12
    assert np.max(np.abs(X[1:] - dirichlet)) < 1e-10


def test_unitary_roundtrip_and_parseval():
    rng = np.random.default_rng(7)
    x = rng.standard_normal(4096) + 1j * rng.standard_normal(4096)
    X = unitary_dft(x)
    assert abs(np.linalg.norm(X) - np.linalg.norm(x)) < 1e-10 * np.linalg.norm(x)
    assert np.max(np.abs(unitary_idft(X) - x)) < 1e-12 * np.linalg.norm(x)


def test_batched_last_axis():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 256)) + 1j * rng.standard_normal((3, 256))
    got = fft_radix2(x)
    for r in range(3):
        assert np.max(np.abs(got[r] - naive_dft(x[r]))) < 1e-11


def test_non_power_of_two_rejected():
    with pytest.raises(ValueError):
        fft_radix2(np.ones(12))
