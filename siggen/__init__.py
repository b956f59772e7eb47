"""Seeded synthetic inputs shared by the oracle and the HIP library's tests.

This module builds input signals only; it holds none of the sparse FFT's
arithmetic.  A planted spectrum (support, values) is drawn from a numpy PCG64
stream, turned into a time signal by an inverse unitary DFT (a library FFT is
fine here: this is input generation, not the method), optionally mixed with
i.i.d. complex Gaussian time-domain noise scaled to an exact tail/head l2
ratio, and cast to the storage dtype.  Both sides then read the same bytes.

Recipes (the workloads of the sparse FFT configurations):
  * support: k distinct frequencies uniform in [0, n)
  * phase:   uniform in [0, 2 pi)
  * magnitude: 1 ("unit") or exp(U[ln lo, ln hi]) ("loguniform", 0.1..10)
  * noise:   complex Gaussian, ||noise||_2 = ratio * ||planted||_2 exactly
             (the unitary DFT preserves the l2 norm, so the ratio holds in
             both time and frequency)
"""
import numpy as np

__all__ = ["planted_spectrum", "time_signal", "planted_signal", "periodic_signal",
           "torch_planted_batch"]


def planted_spectrum(n, k, seed, magnitude="unit", lo=0.1, hi=10.0):
    """(support ascending int64, values complex128) of a k-sparse spectrum."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if k > n:
        raise ValueError("k > n")
    support = np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=k)
    if magnitude == "unit":
        mag = np.ones(k)
    elif magnitude == "loguniform":
        mag = np.exp(rng.uniform(np.log(lo), np.log(hi), size=k))
    elif magnitude == "integer":
        # integer spectra for the paper-literal exact decode: |re|,|im| in 1..4
        re = rng.integers(1, 5, size=k) * rng.choice([-1, 1], size=k)
        im = rng.integers(0, 5, size=k) * rng.choice([-1, 1], size=k)
        return support, (re + 1j * im).astype(np.complex128)
    else:
        raise ValueError(magnitude)
    return support, mag * np.exp(1j * phase)


def time_signal(n, support, values, noise_ratio=0.0, noise_seed=0):
    """x = unitary inverse DFT of the planted spectrum, plus scaled noise (complex128)."""
    X = np.zeros(n, dtype=np.complex128)
    X[support] = values
    x = np.fft.ifft(X) * np.sqrt(n)
    if noise_ratio > 0.0:
        rng = np.random.Generator(np.random.PCG64(noise_seed))
        noise = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        head = np.linalg.norm(values)
        noise *= noise_ratio * head / np.linalg.norm(noise)
        x = x + noise
    return x


def planted_signal(n, k, seed, dtype=np.complex64, magnitude="unit", noise_ratio=0.0):
    """(x in dtype, support, values) from one seed (noise uses seed + 2^32)."""
    support, values = planted_spectrum(n, k, seed, magnitude)
    x = time_signal(n, support, values, noise_ratio, seed + (1 << 32))
    return x.astype(dtype), support, values


def periodic_signal(n, k, seed, dtype=np.complex128):
    """y_t = x_{t mod k} for a random x in C^k (the Section 5 reduction input)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xk = rng.standard_normal(k) + 1j * rng.standard_normal(k)
    return np.tile(xk, n // k).astype(dtype), xk


def torch_planted_batch(n, k, seeds, device, magnitude="unit", noise_ratio=0.0,
                        dtype="complex64", chunk=32):
    """Batch [len(seeds), n] of planted signals built on a torch device.

    Spectra come from planted_spectrum (CPU, cheap); the inverse DFT runs with
    torch.fft on the device in complex128 and is cast to the storage dtype.
    Noise is drawn on the CPU per signal from the same seed rule as
    planted_signal only when noise_ratio > 0 (slow; meant for small batches).
    Returns (x, supports, values).
    """
    import torch

    tdt = getattr(torch, dtype)
    out = torch.empty((len(seeds), n), dtype=tdt, device=device)
    supports, values = [], []
    for c0 in range(0, len(seeds), chunk):
        cs = seeds[c0:c0 + chunk]
        X = torch.zeros((len(cs), n), dtype=torch.complex128, device=device)
        for r, s in enumerate(cs):
            sup, val = planted_spectrum(n, k, int(s), magnitude)
            supports.append(sup)
            values.append(val)
            X[r, torch.from_numpy(sup).to(device)] = torch.from_numpy(val).to(device)
        x = torch.fft.ifft(X, dim=-1, norm="ortho")
        if noise_ratio > 0.0:
            for r, s in enumerate(cs):
                rng = np.random.Generator(np.random.PCG64(int(s) + (1 << 32)))
                noise = rng.standard_normal(n) + 1j * rng.standard_normal(n)
                noise *= noise_ratio * np.linalg.norm(values[c0 + r]) / np.linalg.norm(noise)
                x[r] += torch.from_numpy(noise).to(device)
        out[c0:c0 + len(cs)] = x.to(tdt)
        del X, x
    return out, supports, values
