"""Spectrum permutation, bin/offset maps and HashToBins.

Section 2 (permutation definition):  (P_{sigma,a,b} x)_t = x_{sigma (t - a)} omega^{sigma b t}
and pi_{sigma,b}(i) = sigma (i - b) mod n, so that (P x)^_{pi(i)} = xhat_i omega^{a sigma i}
(the permutation claim).

Section 3 (definitions before the collision claim): the bin of i is
h(i) = round(pi(i) B / n) and its offset is o(i) = pi(i) - h(i) n / B.
Reading: round() is half-up and h is taken mod B, so o(i) lies in
[-n/(2B), n/(2B)); at o = -n/(2B) the window G' is zero, so the tie only
fixes which bin index is reported.

HashToBins (Algorithm 1, computed as in the proof of the HashToBins lemma):
  1. y = G . (P_{sigma,a,b} x) on the window support t in [-w/2, w/2)
  2. v_r = sum_{t = r (mod B)} y_t                     (fold)
  3. u_j = sqrt(n) * FFT_B(v)_j  (= yhat_{jn/B} in the unitary convention)
  4. u_{h(i)} -= G'_{-o(i)} zhat_i omega^{a sigma i}   for i in supp(zhat)
Step 3 scales by sqrt(n) once because G carries no sqrt(n) (window.py).
All index arithmetic is exact integer arithmetic (int64, n <= 2^31).
"""
import numpy as np

from .fft import fft_radix2
from .window import gprime


def _check_n(n):
    if n & (n - 1) or n < 2 or n > (1 << 31):
        raise ValueError("oracle supports power-of-two n in [2, 2^31]")


def perm_position(i, sigma, b, n):
    """pi_{sigma,b}(i) = sigma (i - b) mod n."""
    return (int(sigma) * ((int(i) - int(b)) % n)) % n


def bin_offset(i, sigma, b, n, B):
    """(h(i), o(i)) with h = floor((pi B + n/2) / n) mod B and o = pi - h_unwrapped n/B."""
    p = perm_position(i, sigma, b, n)
    hu = (p * B + n // 2) // n
    return hu % B, p - hu * (n // B)


def omega_pow(e, n):
    """omega^e = exp(-2 pi i (e mod n) / n) for an integer e."""
    return np.exp(-2j * np.pi * float(int(e) % n) / n)


def hash_to_bins_raw(x, sigma, a, b, B, G):
    """Steps 1-3 of HashToBins for one (sigma, a, b); G is window.window_time()."""
    x = np.asarray(x)
    n = x.shape[-1]
    _check_n(n)
    w = len(G)
    t = np.arange(-(w // 2), w - w // 2, dtype=np.int64)
    idx = (int(sigma) * ((t - int(a)) % n)) % n
    c = (int(sigma) * int(b)) % n
    p = (c * (t % n)) % n
    modulation = np.exp(-2j * np.pi * p.astype(np.float64) / n)
    y = G * x[idx].astype(np.complex128) * modulation
    r = t % B
    v = np.bincount(r, weights=y.real, minlength=B) + 1j * np.bincount(r, weights=y.imag, minlength=B)
    return np.sqrt(n) * fft_radix2(v)


def zhat_contribution(i, zi, sigma, a, b, B, n, alpha, delta, kind=0, w=0):
    """(h(i), G'_{-o(i)} zhat_i omega^{a sigma i}) for one entry of zhat (step 4);
    kind, w select the flat window (window.gprime)."""
    h, o = bin_offset(i, sigma, b, n, B)
    g = gprime(-o, n, B, alpha, delta, kind, w)
    return h, g * zi * omega_pow(int(a) * int(sigma) * int(i), n)


def subtract_zhat(u, zhat, sigma, a, b, B, n, alpha, delta, kind=0, w=0):
    """Step 4 of HashToBins, entries of zhat taken in ascending index order."""
    u = np.array(u, dtype=np.complex128)
    for i in sorted(zhat):
        h, c = zhat_contribution(i, zhat[i], sigma, a, b, B, n, alpha, delta, kind, w)
        u[h] -= c
    return u


def hash_to_bins(x, zhat, sigma, a, b, B, G, alpha, delta, kind=0):
    """Full HashToBins(x, zhat, P_{sigma,a,b}, B, delta, alpha)."""
    n = np.asarray(x).shape[-1]
    return subtract_zhat(hash_to_bins_raw(x, sigma, a, b, B, G), zhat, sigma, a, b, B, n, alpha, delta, kind,
                         len(G))
