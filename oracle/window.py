"""Flat window function (G, G') of Section 2 (Definition of a flat window) built
as in Section 7 (the Gaussian-times-boxcar lemma).

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


def window_time(n, B, w, alpha, delta):
    """G_t for t = -w/2, ..., w/2 - 1 (array index u <-> t = u - w/2)."""
    if w % B or w > n:
        raise ValueError("w must be a multiple of B and at most n")
    sigma_g, C = window_shape(n, B, alpha, delta)
    t = np.arange(-(w // 2), w - w // 2, dtype=np.int64)
    return g_star(t, sigma_g, C)


def tail_mass(T, sigma_g, C):
    """sum over |t| >= T of |G*(t)| (both sides).  The Gaussian factor makes
    the terms negligible (< 1e-30 of the first) within 12 sigma_g of T."""
    t = np.arange(T, T + int(12 * sigma_g) + 2, dtype=np.float64)
    return float(2.0 * np.sum(np.abs(g_star(t, sigma_g, C))))


def default_w(n, B, alpha, delta):
    """Smallest multiple of B whose truncation tail sum_{|t|>=w/2}|G*(t)| <= delta,
    or n when no shorter window meets it (then the sparse FFT is not sublinear
    and callers should use a dense transform)."""
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


def phi(x):
    """Standard normal CDF."""
    return 0.5 * math.erfc(-x / math.sqrt(2.0))


def gprime(f, n, B, alpha, delta):
    """G'_f for a signed integer offset f (interpreted mod n).

    In the transition band, with s = |f| / n and Phi(x) = erfc(-x / sqrt 2) / 2,
        Phi(sg (s + C)) - Phi(sg (s - C)) = [erfc(sg (s - C)/sqrt 2) - erfc(sg (s + C)/sqrt 2)] / 2,
    the second form avoiding the cancellation of two values near 1 and being
    exactly even in f.
    """
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
