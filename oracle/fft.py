"""Discrete Fourier transforms written from their definition (Section 2, Notation).

Convention: for x in C^n and omega = exp(-2 pi i / n) the paper's spectrum is
the unitary transform

    xhat_f = n^{-1/2} * sum_j omega^{f j} x_j .

Internally the oracle works with the unnormalised transform
X_f = sum_j omega^{f j} x_j and applies n^{-1/2} where the paper does.
No numpy.fft is used by the method; the radix-2 FFT below is our own.
"""
import numpy as np


def naive_dft(x):
    """Unnormalised DFT by the O(n^2) sum (intended for n <= 4096).

    The exponent f*j is reduced mod n in exact integers before the complex
    exponential, so each matrix entry is one correctly rounded root of unity.
    """
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    j = np.arange(n, dtype=np.int64)
    fj = np.outer(j, j) % n
    W = np.exp(-2j * np.pi * fj.astype(np.float64) / n)
    return x @ W.T


def _bit_reverse_permutation(n):
    m = n.bit_length() - 1
    idx = np.arange(n, dtype=np.int64)
    rev = np.zeros(n, dtype=np.int64)
    for bit in range(m):
        rev |= ((idx >> bit) & 1) << (m - 1 - bit)
    return rev


def fft_radix2(x):
    """Unnormalised DFT of the last axis by iterative radix-2 decimation in time.

    n must be a power of two (Section 2, Assumptions).  Stage s combines pairs
    of length-(size/2) transforms with twiddles exp(-2 pi i k / size).
    """
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    if n & (n - 1):
        raise ValueError("fft_radix2 needs a power-of-two length")
    a = x[..., _bit_reverse_permutation(n)]
    lead = a.shape[:-1]
    size = 2
    while size <= n:
        half = size // 2
        tw = np.exp(-2j * np.pi * np.arange(half, dtype=np.float64) / size)
        a = a.reshape(lead + (n // size, size))
        even = a[..., :half]
        odd = a[..., half:] * tw
        a = np.concatenate([even + odd, even - odd], axis=-1).reshape(lead + (n,))
        size *= 2
    return a


def unitary_dft(x):
    """The paper's xhat = n^{-1/2} * X."""
    x = np.asarray(x, dtype=np.complex128)
    return fft_radix2(x) / np.sqrt(x.shape[-1])


def unitary_idft(xhat):
    """Inverse of unitary_dft: x_j = n^{-1/2} sum_f omega^{-f j} xhat_f."""
    xhat = np.asarray(xhat, dtype=np.complex128)
    return np.conj(fft_radix2(np.conj(xhat))) / np.sqrt(xhat.shape[-1])
