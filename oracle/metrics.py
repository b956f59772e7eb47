"""Error measures of the l2/l2 guarantee (Section 1, eq. (1); Err of Section 4,
formal definitions).

Err(xhat, k) = min over k-sparse y of ||xhat - y||_2 = sqrt(sum of all but the
k largest |xhat_f|^2).  The spectrum comes from the oracle's own FFT of the
very bytes the sparse FFT read.
"""
import numpy as np

from .fft import unitary_dft


def err_k(xhat, k):
    mag2 = np.sort(np.abs(np.asarray(xhat)) ** 2)
    return float(np.sqrt(np.sum(mag2[: max(0, len(mag2) - k)])))


def sparse_to_dense(n, indices, values):
    out = np.zeros(n, dtype=np.complex128)
    out[np.asarray(indices, dtype=np.int64)] = values
    return out


def l2_error(xhat, indices, values):
    """||xhat - xhat'||_2 for a sparse estimate."""
    diff = np.asarray(xhat, dtype=np.complex128).copy()
    diff[np.asarray(indices, dtype=np.int64)] -= values
    return float(np.linalg.norm(diff))


def l2l2_ratio(x, k, indices, values):
    """(||xhat - xhat'||_2 / Err(xhat, k), Err) with xhat the unitary DFT of x."""
    xhat = unitary_dft(np.asarray(x, dtype=np.complex128))
    e = err_k(xhat, k)
    num = l2_error(xhat, indices, values)
    return (num / e if e > 0 else (0.0 if num == 0 else np.inf)), e
