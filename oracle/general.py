"""General (noisy) k-sparse recovery: Algorithms 2 and 3 (SparseFFT,
EstimateValues, LocateSignal, LocateInner) in FP64.

SparseFFT (Algorithm 2), practical schedule (reading of the round parameters of
the general-case theorem, whose constants are only asymptotic): round r uses
    k_r = max(1, k >> 2r)   (the "k -> k/4" step of the Section 4 intuition),
    B_r = max(B >> r, 4 k_r rounded up to a power of two, b_min), capped at B,
    w_r = w B_r / B,
(b_min = B holds B and w fixed, the comparison the schedule is measured
against),
and does  L = LocateSignal(x, zhat, B_r),  zhat += EstimateValues(x, zhat, 3 k_r, L, B_r).

LocateSignal (Algorithm 3): one (sigma, b) per round; regions start at
l_j = j n / B - n / (2B) with width W = n / B (bins are centred at j n / B, so
the regions are taken centred and half-open, [l, l + W)); LocateInner runs while
W > 1 and each level shrinks W by t' = t / 4.  The result is
L = { sigma^{-1} ceil(l_j) + b  mod n } over the bins whose regions survive.

LocateInner (Algorithm 3): for each of R_loc measurements draw a and
beta in [ceil(s n t / (4W)), floor(s n t / (2W))], hash at a and a + beta
(the same sigma, b), and let c_j be the phase of u_j / u'_j.  Region q of bin
j (centre m = l_j + (q - 1/2) W / t) gets a vote when the circular distance
between beta * 2 pi (m + sigma b) / n and c_j is below s pi.  The new start is
l_j + (min Q* - 1) W / t with Q* = {q : votes > R_loc / 2}; an empty Q* drops
the bin.  LocateSignal passes b (not beta) to LocateInner.  Region
coordinates are dyadic, so they are held as integers with FRAC_BITS
fractional bits and the angle beta (m + sigma b) mod n is reduced exactly.

EstimateValues (Algorithm 2): R_est fresh (sigma_e, a_e, b_e); for i in L the
estimates e = u_{h_e(i)} omega^{-a_e sigma_e i} / G'_{-o_e(i)} over the
measurements with G' >= g_min; w_i is the coordinate-wise median; the k'
entries of largest |w_i| are kept (ties: smaller index).  Reading: the division
by G' and the g_min filter are added (the paper's estimate omits G', which
biases it whenever the offset is large).

Final FP64 re-estimation: every zhat entry is re-estimated from all stored
EstimateValues measurements, with the other zhat entries of the same bin
subtracted, resolved in passes as in exact mode (reestimate.py: entries alone
in a bin first, then entries whose bin neighbours are resolved); the output
is the top-cap entries by magnitude, ascending index.

Parity unpinned: which noisy heads a run finds has no closed form; the oracle
run itself and the statistical l2/l2 guarantee of Section 1 eq. (1) are what
pin it (tests/test_oracle_general.py).
"""
import math
from dataclasses import dataclass, field

import numpy as np

from .hashing import bin_offset, hash_to_bins_raw, omega_pow, subtract_zhat
from .params import SfftParams, complex_median
from .reestimate import peel_reestimate
from .rng import LEVEL_EST, draw_a, draw_b, draw_beta, draw_sigma, inverse_mod
from .window import gprime, window_time

TWO_PI = 2.0 * math.pi
FRAC_BITS = 8


def round_schedule(p: SfftParams, r):
    """(k_r, B_r, w_r) of SparseFFT round r; b_min > 0 is a further floor on
    B_r (b_min = B keeps B and w fixed in every round)."""
    k_r = max(1, p.k >> (2 * r))
    floor = 1
    while floor < 4 * k_r:
        floor <<= 1
    B_r = min(p.B, max(p.B >> r, floor, p.b_min))
    return k_r, B_r, p.w * B_r // p.B


def level_widths(n, B, t):
    """Region widths W (in FRAC_BITS fixed point) of the LocateInner levels."""
    scale = 1 << FRAC_BITS
    W = (n // B) * scale
    out = []
    while W > scale:
        out.append(W)
        W = W * 4 // t
    return out


def beta_range(n, W_fp, t, s):
    """Integer beta range [ceil(s n t / (4W)), floor(s n t / (2W))], W real = W_fp / 2^FRAC_BITS."""
    W = W_fp / float(1 << FRAC_BITS)
    lo = math.ceil(s * n * t / (4.0 * W))
    hi = math.floor(s * n * t / (2.0 * W))
    lo = max(lo, 1)
    return lo, max(hi, lo)


@dataclass
class GeneralResult:
    indices: np.ndarray
    values: np.ndarray
    zhat: dict
    located: list = field(default_factory=list)      # L per round (sorted)
    estimated: list = field(default_factory=list)    # accepted dict per round
    est_raw: list = field(default_factory=list)      # (sigma, a, b, B_r, u_raw)
    vote_margin: float = math.inf                    # | dist - s pi | over all votes
    select_margin: float = math.inf                  # top-k' boundary gap
    trace: list = None                               # per level (W, l, dist per rep, winners)


def phase_of_ratio(u, u2):
    """phi(u / u2) in [0, 2 pi), computed as the argument of u * conj(u2)."""
    z = u * np.conj(u2)
    ph = np.arctan2(z.imag, z.real)
    return np.where(ph < 0.0, ph + TWO_PI, ph)


def locate_signal(x, zhat, r, B, G, p: SfftParams, res: GeneralResult):
    n = p.n
    # beta * (angle numerator) must stay below 2^63 in int64
    assert n <= (1 << 26), "oracle general mode supports n <= 2^26"
    scale = 1 << FRAC_BITS
    mod = n * scale
    sigma = draw_sigma(p.seed, n, r, 0, 0)
    b = draw_b(p.seed, n, r, 0, 0)
    sb = (sigma * b) % n
    j = np.arange(B, dtype=np.int64)
    l = ((j * (n // B) - n // (2 * B)) * scale) % mod
    alive = np.ones(B, dtype=bool)
    qs = np.arange(1, p.t + 1, dtype=np.int64)
    for D, W in enumerate(level_widths(n, B, p.t), start=1):
        lo, hi = beta_range(n, W, p.t, p.s)
        votes = np.zeros((B, p.t), dtype=np.int64)
        dists = []
        # region centres m_{j,q} = l_j + (q - 1/2) W / t, in fixed point
        half_step = W // (2 * p.t)
        M = (l[:, None] + (2 * qs[None, :] - 1) * half_step) % mod
        for q in range(p.R_loc):
            a = draw_a(p.seed, n, r, D, q)
            beta = draw_beta(p.seed, lo, hi, r, D, q)
            u = hash_to_bins(x, zhat, sigma, a, b, B, G, p)
            u2 = hash_to_bins(x, zhat, sigma, a + beta, b, B, G, p)
            c = phase_of_ratio(u, u2)
            num = (beta * ((M + sb * scale) % mod)) % mod
            ang = TWO_PI * num.astype(np.float64) / float(mod)
            d = np.abs(ang - c[:, None])
            dist = np.minimum(d, TWO_PI - d)
            res.vote_margin = min(res.vote_margin, float(np.min(np.abs(dist - p.s * math.pi)[alive])) if alive.any() else math.inf)
            votes += dist < p.s * math.pi
            dists.append(dist)
        winners = votes > (p.R_loc / 2.0)
        if res.trace is not None:
            res.trace.append((W, l.copy(), dists, winners))
        has = winners.any(axis=1)
        first = np.argmax(winners, axis=1)          # index of min q in Q* (0-based)
        step = W // p.t
        l = np.where(has, (l + first * step) % mod, l)
        alive &= has
    sigma_inv = inverse_mod(sigma, n)
    pos = ((l + scale - 1) // scale) % n            # ceil(l_j)
    L = sorted({int((sigma_inv * int(pp)) % n + b) % n for pp, ok in zip(pos, alive) if ok})
    return L


def hash_to_bins(x, zhat, sigma, a, b, B, G, p):
    n = p.n
    raw = hash_to_bins_raw(x, sigma, a % n, b, B, G)
    return subtract_zhat(raw, zhat, sigma, a % n, b, B, n, p.alpha, p.delta, p.window, len(G))


def estimate_values(x, zhat, r, kprime, L, B, G, p: SfftParams, res: GeneralResult):
    n = p.n
    meas = []
    for e in range(p.R_est):
        sigma = draw_sigma(p.seed, n, r, LEVEL_EST, e)
        a = draw_a(p.seed, n, r, LEVEL_EST, e)
        b = draw_b(p.seed, n, r, LEVEL_EST, e)
        raw = hash_to_bins_raw(x, sigma, a, b, B, G)
        res.est_raw.append((sigma, a, b, B, raw))
        meas.append((sigma, a, b, subtract_zhat(raw, zhat, sigma, a, b, B, n, p.alpha, p.delta, p.window, len(G))))
    w = {}
    for i in L:
        vals = []
        for sigma, a, b, u in meas:
            h, o = bin_offset(i, sigma, b, n, B)
            g = gprime(-o, n, B, p.alpha, p.delta, p.window, len(G))
            if g < p.g_min:
                continue
            vals.append(u[h] * omega_pow(-(a * sigma * i), n) / g)
        if vals:
            w[i] = complex_median(vals)
    order = sorted(w, key=lambda i: (-abs(w[i]), i))
    if len(order) > kprime:
        res.select_margin = min(res.select_margin, abs(abs(w[order[kprime - 1]]) - abs(w[order[kprime]])))
    return {i: w[i] for i in order[:kprime]}


def reestimate_general(zhat, est_raw, p: SfftParams):
    """FP64 median re-estimation of every zhat entry over all stored
    EstimateValues measurements, resolved in passes by
    reestimate.peel_reestimate (term coefficient G' omega^{a sigma i})."""
    n = p.n
    meas = []
    for sigma, a, b, B, raw in est_raw:
        terms = {}
        for i in zhat:
            h, o = bin_offset(i, sigma, b, n, B)
            g = gprime(-o, n, B, p.alpha, p.delta, p.window, p.w // p.B * B)
            terms[i] = (h, g, g * omega_pow(a * sigma * i, n))
        meas.append((raw, terms))
    return peel_reestimate(zhat, meas, p.g_min)


def sparse_fft(x, p: SfftParams) -> GeneralResult:
    x = np.asarray(x)
    n = x.shape[-1]
    assert n == p.n
    res = GeneralResult(np.zeros(0, np.int64), np.zeros(0, np.complex128), {})
    zhat = {}
    for r in range(p.rounds):
        k_r, B_r, w_r = round_schedule(p, r)
        G = window_time(n, B_r, w_r, p.alpha, p.delta, p.window)
        L = locate_signal(x, zhat, r, B_r, G, p, res)
        res.located.append(L)
        upd = estimate_values(x, zhat, r, 3 * k_r, L, B_r, G, p, res)
        res.estimated.append(upd)
        for i in sorted(upd):
            zhat[i] = zhat.get(i, 0.0 + 0.0j) + upd[i]
    res.zhat = dict(zhat)
    values = reestimate_general(zhat, res.est_raw, p)
    order = sorted(values, key=lambda i: (-abs(values[i]), i))
    if len(order) > p.out_cap:
        res.select_margin = min(res.select_margin,
                                abs(abs(values[order[p.out_cap - 1]]) - abs(values[order[p.out_cap]])))
    keep = sorted(order[:p.out_cap])
    res.indices = np.array(keep, dtype=np.int64)
    res.values = np.array([values[i] for i in keep], dtype=np.complex128)
    return res
