"""Flat window function (G, G') of Section 2 (Definition of a flat window) built
as in Section 7 (the Gaussian-times-boxcar lemma), or (kind 1) from a
Kaiser-Bessel taper of the same ideal low-pass (kaiser_* below).

Continuous prototype (Section 7): D is a Gaussian whose transform has standard
deviation 1/sigma_g, and F is the inverse transform of a boxcar of half-width C,
so that

    G*(t)     = exp(-2 pi^2 t^2 / sigma_g^2) * sin(2 pi C t) / (pi t),  G*(0) = 2C
    Ghat*(s)  = Phi(sigma_g (s + C)) - Phi(sigma_g (s - C))

with C = (1 - alpha/2)/(2B) and sigma_g = (4B/alpha) sqrt(2 ln(3/delta)).
Reading of the parameter choice at the end of the Section 7 lemma: the paper
takes sigma_g = (4B/alpha) sqrt(2 log(n/delta)) after replacing delta by
delta/n, a step that only absorbs the sqrt(n) its normalisation puts into G
(its (8 sqrt(n) + 6) delta bound).  Here G carries no sqrt(n), so the lemma's
own requirement - Phi below delta beyond sqrt(2 log(3/delta)) (the CDF claim,
item 4) - is met with log(3/delta); the result still satisfies
||Ghat - G'||_inf < delta (pinned by test) with a shorter window.  Reading of
the garbled passages: F(t) is 2C*sinc(2Ct), D(t) is the Gaussian above, and
the G' argument is sigma_g*(f/n +- C).

Discrete window: G_t = G*(t) for integer t in [-w/2, w/2), zero elsewhere.
The paper folds sqrt(n) into G; we instead apply sqrt(n) once to the bins
(hashing.py), which gives the same bins.  With this scaling the unitary-DFT
identity of the HashToBins lemma (Section 3) holds with Ghat(f) ~= Ghat*(f/n)
(Poisson summation, the continuous-DFT claim of Section 7).

G'_f (Section 2 definition, Section 7 evaluation):
    1                                  if |f| <= (1 - alpha) n / (2B)
    0                                  if |f| >= n / (2B)
    Phi(sg (f/n + C)) - Phi(sg (f/n - C)) otherwise (evaluated at |f|)
with Phi the standard normal CDF, Phi(x) = erfc(-x / sqrt 2) / 2.
"""
import functools
import math

import numpy as np


def window_shape(n, B, alpha, delta):
    """(sigma_g, C) of the Section 7 lemma (n enters only through the caller's
    delta; see the module docstring)."""
    sigma_g = (4.0 * B / alpha) * math.sqrt(2.0 * math.log(3.0 / delta))
    C = (1.0 - alpha / 2.0) / (2.0 * B)
    return sigma_g, C


def g_star(t, sigma_g, C):
    """Continuous window G*(t) = Gaussian(t) * sin(2 pi C t)/(pi t), G*(0) = 2C."""
    t = np.asarray(t, dtype=np.float64)
    gauss = np.exp(-2.0 * math.pi ** 2 * t * t / (sigma_g * sigma_g))
    with np.errstate(invalid="ignore", divide="ignore"):
        box = np.where(t == 0.0, 2.0 * C, np.sin(2.0 * math.pi * C * t) / (math.pi * t))
    return gauss * box


def window_time(n, B, w, alpha, delta, kind=0):
    """G_t for t = -w/2, ..., w/2 - 1 (array index u <-> t = u - w/2)."""
    if w % B or w > n:
        raise ValueError("w must be a multiple of B and at most n")
    if kind == 1:
        return kaiser_time(n, B, w, alpha, delta)
    sigma_g, C = window_shape(n, B, alpha, delta)
    t = np.arange(-(w // 2), w - w // 2, dtype=np.int64)
    return g_star(t, sigma_g, C)


def tail_mass(T, sigma_g, C):
    """sum over |t| >= T of |G*(t)| (both sides).  The Gaussian factor makes
    the terms negligible (< 1e-30 of the first) within 12 sigma_g of T."""
    t = np.arange(T, T + int(12 * sigma_g) + 2, dtype=np.float64)
    return float(2.0 * np.sum(np.abs(g_star(t, sigma_g, C))))


def default_w(n, B, alpha, delta, kind=0):
    """Smallest multiple of B whose truncation tail sum_{|t|>=w/2}|G*(t)| <= delta,
    or n when no shorter window meets it (then the sparse FFT is not sublinear
    and callers should use a dense transform).  Kind 1: kaiser_w."""
    if kind == 1:
        return kaiser_w(n, B, alpha, delta)
    sigma_g, C = window_shape(n, B, alpha, delta)
    lo, hi = 1, n // B            # w = m B; tail decreasing in m
    if tail_mass(hi * B // 2, sigma_g, C) > delta:
        return n
    while lo < hi:
        mid = (lo + hi) // 2
        if tail_mass(mid * B // 2, sigma_g, C) <= delta:
            hi = mid
        else:
            lo = mid + 1
    return lo * B


# ------------------------------------------------------------------ kind 1 --
# Section 2 defines a flat window by its properties: G' is 1 on
# |f| <= (1 - alpha) n / (2B), 0 on |f| >= n / (2B), and ||Ghat - G'||_inf < delta;
# the Section 7 lemma shows one exists (the Gaussian construction above).
# Kind 1 meets the same definition with a shorter support: the ideal
# low-pass sin(2 pi C t) / (pi t) (the same C) tapered by the Kaiser-Bessel
# window I0(beta sqrt(1 - (2t/w)^2)) / I0(beta), with Kaiser's empirical rules
# (J. F. Kaiser, "Nonrecursive digital filter design using the I0-sinh window
# function", 1974) for a ripple of delta / 2 on both sides of a transition
# band of alpha / (2B) cycles per sample:
#     A = -20 log10(delta / 2),  beta = 0.1102 (A - 8.7)  (A > 50),
#     length N = (A - 7.95) / (14.36 alpha / (2B)) + 1,  w = N rounded up to a
#     multiple of B (at most n).
# G' in the transition band is the window's own response there,
#     G'_f = sum_t G_t cos(2 pi f t / n)  (clamped to [0, 1]),
# the real part of its DTFT at integer f, so ||Ghat - G'|| is the ripple
# outside the band plus the response's imaginary part (from the one unpaired
# end sample t = -w/2), both below delta (pinned by test).


def bessel_i0(x):
    """Modified Bessel function I0 by its power series sum (x/2)^2k / (k!)^2."""
    x = np.asarray(x, dtype=np.float64)
    q = (x * 0.5) ** 2
    term = np.ones_like(x)
    total = np.ones_like(x)
    for k in range(1, 200):
        term = term * q / (k * k)
        total = total + term
        if np.all(term <= 1e-17 * total):
            break
    return total


def kaiser_beta(delta):
    """Kaiser's shape parameter for a ripple of delta / 2."""
    A = -20.0 * math.log10(delta / 2.0)
    if A > 50.0:
        return 0.1102 * (A - 8.7)
    if A >= 21.0:
        return 0.5842 * (A - 21.0) ** 0.4 + 0.07886 * (A - 21.0)
    return 0.0


def kaiser_w(n, B, alpha, delta):
    """Kaiser's length rule for the transition band alpha / (2B), rounded up to
    a multiple of B, at most n."""
    A = -20.0 * math.log10(delta / 2.0)
    N = (A - 7.95) / (14.36 * alpha / (2.0 * B)) + 1.0
    return min(n, int(math.ceil(N / B)) * B)


def kaiser_time(n, B, w, alpha, delta):
    """G_t for t = -w/2, ..., w/2 - 1 of the kind-1 window."""
    C = (1.0 - alpha / 2.0) / (2.0 * B)
    t = np.arange(-(w // 2), w - w // 2, dtype=np.int64).astype(np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        box = np.where(t == 0.0, 2.0 * C, np.sin(2.0 * math.pi * C * t) / (math.pi * t))
    r = 2.0 * t / w
    beta = kaiser_beta(delta)
    return box * bessel_i0(beta * np.sqrt(np.maximum(1.0 - r * r, 0.0))) / bessel_i0(np.float64(beta))


@functools.lru_cache(maxsize=64)
def _kaiser_window(n, B, w, alpha, delta):
    G = kaiser_time(n, B, w, alpha, delta)
    t = np.arange(-(w // 2), w - w // 2, dtype=np.int64)
    return G, t


@functools.lru_cache(maxsize=64)
def _kaiser_gprime_table(n, B, w, alpha, delta):
    """G'_f of the kind-1 window for f = 0 .. n/(2B): the same sum as
    kaiser_gprime describes, evaluated once for every f of the band."""
    G, t = _kaiser_window(n, B, w, alpha, delta)
    f = np.arange(n // (2 * B) + 1, dtype=np.int64)
    out = np.where(f * 2 * B <= (1.0 - alpha) * n, 1.0, 0.0)
    band = np.nonzero((f * 2 * B > (1.0 - alpha) * n) & (f * 2 * B < n))[0]
    step = max(1, (1 << 22) // max(w, 1))
    for q in range(0, len(band), step):
        fs = f[band[q:q + step]]
        ang = 2.0 * math.pi * ((fs[:, None] * t[None, :]) % n).astype(np.float64) / n
        out[band[q:q + step]] = np.clip(np.sum(G[None, :] * np.cos(ang), axis=1), 0.0, 1.0)
    return out


def kaiser_gprime(f, n, B, w, alpha, delta):
    """G'_f of the kind-1 window (signed integer f, taken mod n): 1 in the
    pass band, 0 from n/(2B) on, sum_t G_t cos(2 pi f t / n) clamped to
    [0, 1] in between (tabulated per window by _kaiser_gprime_table)."""
    f = int(f) % n
    if f >= n // 2:
        f -= n
    af = abs(f)
    if af * 2 * B <= (1.0 - alpha) * n:
        return 1.0
    if af * 2 * B >= n:
        return 0.0
    return float(_kaiser_gprime_table(n, B, w, alpha, delta)[af])


def phi(x):
    """Standard normal CDF."""
    return 0.5 * math.erfc(-x / math.sqrt(2.0))


def gprime(f, n, B, alpha, delta, kind=0, w=0):
    """G'_f for a signed integer offset f (interpreted mod n); kind 1 is the
    Kaiser window of length w (kaiser_gprime), kind 0 the Gaussian one:

    In the transition band, with s = |f| / n and Phi(x) = erfc(-x / sqrt 2) / 2,
        Phi(sg (s + C)) - Phi(sg (s - C)) = [erfc(sg (s - C)/sqrt 2) - erfc(sg (s + C)/sqrt 2)] / 2,
    the second form avoiding the cancellation of two values near 1 and being
    exactly even in f.
    """
    if kind == 1:
        return kaiser_gprime(f, n, B, w, alpha, delta)
    f = int(f) % n
    if f >= n // 2:
        f -= n
    af = abs(f)
    if af * 2 * B <= (1.0 - alpha) * n:
        return 1.0
    if af * 2 * B >= n:
        return 0.0
    sigma_g, C = window_shape(n, B, alpha, delta)
    s = af / n
    r2 = math.sqrt(2.0)
    return 0.5 * (math.erfc(sigma_g * (s - C) / r2) - math.erfc(sigma_g * (s + C) / r2))
