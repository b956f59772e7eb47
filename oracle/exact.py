"""Exactly k-sparse recovery: Algorithm 1 (NoiselessSparseFFT) in FP64.

Per round r (NoiselessSparseFFTInner), with B_r = max(B >> r, b_min) bins and a
w_r = w B_r / B window (params.round_bins):
  * draw sigma odd and b uniform (rng.py, counter (r, 0, 0));
  * u  = HashToBins(x, zhat, P_{sigma,0,b}),  u' = HashToBins(x, zhat, P_{sigma,1,b});
  * J  = { j : |u_j| > theta };  stop after `patience` consecutive rounds with
    J empty, or after `stop_patience` once `stop_count` (> 0) entries of zhat
    exceed theta/2 in magnitude (or after `rounds` rounds);
  * for j in J (with ratio_tol > 0, only bins where |u'_j|^2 is within that
    fraction of |u_j|^2): the phase of u_j / u'_j equals 2 pi sigma i / n for an isolated
    coefficient (the exact-estimation lemma of Section 3), so
        p = round(phi(u_j / u'_j) n / (2 pi)) mod n,   i = sigma^{-1} p mod n;
    (with refine_shift = A > 0 a third hashing u_A = HashToBins(x, zhat,
    P_{sigma,A,b}) refines p: the candidate c within refine_window of p whose
    angle 2 pi (A c mod n) / n is nearest the phase of u_j / u_A,j);
    accept i only if h(i) = j and G'_{-o(i)} >= g_min, with value
        v = u_j / G'_{-o(i)}
    (the HashToBins lemma with a single term; equals the paper's round(u_j)
    when G' = 1 and the spectrum is integral);
  * zhat_i += v.
Readings: phi is taken in [0, 2 pi); round() is half-up; the bin check keeps
every accepted i tied to the one bin that can hold it, so the writes of one
round never conflict.  The phase is computed as the argument of
u_j * conj(u'_j), which has the phase of u_j / u'_j.

After the last round the values are re-estimated in FP64 (reestimate.py):
for each i in supp(zhat) and each round r whose window value
G'_{-o_r(i)} >= g_min,
    e_r = (u_raw_r[h_r(i)] - sum_{i' != i, h_r(i') = h_r(i)} G'_{-o_r(i')} v_{i'}) / G'_{-o_r(i)}
(the EstimateValues estimate of Algorithm 2 with a = 0, applied to x minus the
other recovered coefficients), and the value is a coordinate-wise median of
the e_r.  Entries are resolved in passes: first those alone in their bin in
some round (the no-collision case of the estimation lemmas), then those with
a round whose other bin members are all resolved, subtracting the resolved
values v_{i'}; so the window leakage a decoded value picked up from a
neighbour that was found later does not pass into the estimates.  The
output keeps entries with |value| > theta/2, at most cap of them (largest
magnitude first, then smaller index), in ascending index order.

The paper-literal variant (params.literal) keeps v = round(u_j) and writes
without the bin/window checks; conflicting writes keep the larger |u_j|,
then the smaller j.
"""
import math
from dataclasses import dataclass, field

import numpy as np

from .hashing import bin_offset, hash_to_bins_raw, subtract_zhat
from .params import SfftParams
from .reestimate import peel_reestimate
from .rng import draw_b, draw_sigma, inverse_mod
from .window import gprime, window_time

TWO_PI = 2.0 * math.pi


@dataclass
class Margins:
    """Smallest distance of any floating-point decision from its threshold."""

    threshold: float = math.inf   # | |u_j| - theta |
    rounding: float = math.inf    # distance of phi n / 2pi from a half-integer
    gmin: float = math.inf        # | G' - g_min | for decoded candidates
    output: float = math.inf      # | |value| - theta/2 |
    ratio: float = math.inf       # | ||u'|^2 - |u|^2| / |u|^2 - ratio_tol | when the check is on
    refine: float = math.inf      # gap between the best and second-best refinement candidates (radians)

    def smallest(self):
        return min(self.threshold, self.rounding, self.gmin, self.output, self.ratio, self.refine)


@dataclass
class ExactResult:
    indices: np.ndarray
    values: np.ndarray
    rounds_used: int
    truncated: bool
    zhat_decoded: dict
    round_log: list = field(default_factory=list)   # (|J|, accepted) per round
    raw: list = field(default_factory=list)         # (sigma, b, u0_raw, u1_raw) per round
    raw_refine: list = field(default_factory=list)  # u_A raw bins per round (refine_shift > 0)
    margins: Margins = field(default_factory=Margins)


def refine_position(p0, phase_a, A, n, E, margins: Margins):
    """The position c in [p0 - E, p0 + E] whose angle 2 pi (A c mod n) / n is
    nearest (circularly) to phase_a, the phase of u / u_A; ties keep the
    smaller c.  An isolated coefficient at permuted position p has
    u_A = u omega^{A p} (the exact-estimation lemma at shift A), so this
    angle is exact in integers and the phase pins p once the coarse error
    is within E and A (2E + 1) < n."""
    best, bestd, second = None, math.inf, math.inf
    for c in range(p0 - E, p0 + E + 1):
        ang = TWO_PI * ((A * c) % n) / n
        d = abs(ang - phase_a) % TWO_PI
        d = min(d, TWO_PI - d)
        if d < bestd:
            second, bestd, best = bestd, d, c
        elif d < second:
            second = d
    margins.refine = min(margins.refine, second - bestd)
    return best % n


def decode_bin(u0j, u1j, j, sigma, sigma_inv, b, B, p: SfftParams, margins: Margins, alpha=None, uAj=None, w=0):
    """Location and value of bin j of a B-bin hashing; returns (i, v) or None.
    With ratio_tol > 0 a bin whose two hashings differ in magnitude by more
    than that fraction is not decoded: an isolated coefficient gives
    u'_j = u_j omega^{sigma i} (the exact-estimation lemma), equal in
    magnitude, while a bin shared by several coefficients almost never does.
    With refine_shift > 0 the position from the pair's phase is refined by the
    third hashing uAj (refine_position)."""
    n = p.n
    if p.ratio_tol > 0.0:
        m0 = u0j.real * u0j.real + u0j.imag * u0j.imag
        m1 = u1j.real * u1j.real + u1j.imag * u1j.imag
        margins.ratio = min(margins.ratio, abs(abs(m1 - m0) / m0 - p.ratio_tol))
        if abs(m1 - m0) > p.ratio_tol * m0:
            return None
    z = u0j * np.conj(u1j)
    phi = math.atan2(z.imag, z.real)
    if phi < 0.0:
        phi += TWO_PI
    q = phi / TWO_PI * n
    margins.rounding = min(margins.rounding, abs(q - math.floor(q) - 0.5))
    pos = int(math.floor(q + 0.5)) % n
    if p.refine_shift:
        zA = u0j * np.conj(uAj)
        phA = math.atan2(zA.imag, zA.real)
        if phA < 0.0:
            phA += TWO_PI
        pos = refine_position(pos, phA, p.refine_shift, n, p.refine_window, margins)
    i = (sigma_inv * pos) % n
    if p.literal:
        return i, complex(round(u0j.real), round(u0j.imag))
    h, o = bin_offset(i, sigma, b, n, B)
    if h != j:
        return None
    g = gprime(-o, n, B, p.alpha if alpha is None else alpha, p.delta, p.window, w)
    margins.gmin = min(margins.gmin, abs(g - p.g_min))
    if g < p.g_min:
        return None
    return i, u0j / g


def noiseless_sparse_fft(x, p: SfftParams) -> ExactResult:
    x = np.asarray(x)
    n = x.shape[-1]
    assert n == p.n
    zhat = {}
    res = ExactResult(np.zeros(0, np.int64), np.zeros(0, np.complex128), 0, False, {})
    rounds_used = p.rounds
    empty_run = 0
    for r in range(p.rounds):
        sigma = draw_sigma(p.seed, n, r)
        b = draw_b(p.seed, n, r)
        sigma_inv = inverse_mod(sigma, n)
        Br, wr = p.round_bins(r)
        ar = p.round_alpha(r)
        G = window_time(n, Br, wr, ar, p.delta, p.window)
        u0_raw = hash_to_bins_raw(x, sigma, 0, b, Br, G)
        u1_raw = hash_to_bins_raw(x, sigma, 1, b, Br, G)
        res.raw.append((sigma, b, u0_raw, u1_raw))
        u0 = subtract_zhat(u0_raw, zhat, sigma, 0, b, Br, n, ar, p.delta, p.window, wr)
        u1 = subtract_zhat(u1_raw, zhat, sigma, 1, b, Br, n, ar, p.delta, p.window, wr)
        uA = None
        if p.refine_shift:
            uA_raw = hash_to_bins_raw(x, sigma, p.refine_shift, b, Br, G)
            res.raw_refine.append(uA_raw)
            uA = subtract_zhat(uA_raw, zhat, sigma, p.refine_shift, b, Br, n, ar, p.delta, p.window, wr)
        mag = np.abs(u0)
        res.margins.threshold = min(res.margins.threshold, float(np.min(np.abs(mag - p.theta))))
        J = [j for j in range(Br) if mag[j] > p.theta]
        if not J:
            res.round_log.append((0, 0))
            empty_run += 1
            found = sum(1 for v in zhat.values() if abs(v) > 0.5 * p.theta)
            if empty_run >= p.patience or (p.stop_count > 0 and empty_run >= p.stop_patience and
                                           found >= p.stop_count):
                rounds_used = r + 1
                break
            continue
        empty_run = 0
        updates = {}
        best = {}
        for j in J:
            got = decode_bin(u0[j], u1[j], j, sigma, sigma_inv, b, Br, p, res.margins, ar,
                             None if uA is None else uA[j], wr)
            if got is None:
                continue
            i, v = got
            if p.literal and i in updates:
                # conflicting writes: larger |u_j| wins, then the smaller j
                if (mag[j], -j) <= best[i]:
                    continue
            updates[i] = v
            best[i] = (mag[j], -j)
        for i in sorted(updates):
            zhat[i] = zhat.get(i, 0.0 + 0.0j) + updates[i]
        res.round_log.append((len(J), len(updates)))
    res.rounds_used = rounds_used
    res.zhat_decoded = dict(zhat)
    values = reestimate(zhat, res.raw[:rounds_used], p) if not p.literal else dict(zhat)
    _finish(res, values, p)
    return res


def reestimate(zhat, raw, p: SfftParams):
    """FP64 median re-estimation of every zhat entry over the given rounds
    (shift a = 0 of each round's pair), resolved in passes by
    reestimate.peel_reestimate."""
    n = p.n
    meas = []
    for r, (sigma, b, u0_raw, _u1) in enumerate(raw):
        B, wr = p.round_bins(r)
        ar = p.round_alpha(r)
        terms = {}
        for i in zhat:
            h, o = bin_offset(i, sigma, b, n, B)
            g = gprime(-o, n, B, ar, p.delta, p.window, wr)
            terms[i] = (h, g, g)
        meas.append((u0_raw, terms))
    return peel_reestimate(zhat, meas, p.g_min)


def _finish(res: ExactResult, values: dict, p: SfftParams):
    half = 0.5 * p.theta
    kept = []
    for i, v in values.items():
        res.margins.output = min(res.margins.output, abs(abs(v) - half))
        if abs(v) > half:
            kept.append((i, v))
    cap = p.out_cap
    if len(kept) > cap:
        kept.sort(key=lambda e: (-abs(e[1]), e[0]))
        kept = kept[:cap]
        res.truncated = True
    kept.sort(key=lambda e: e[0])
    res.indices = np.array([e[0] for e in kept], dtype=np.int64)
    res.values = np.array([e[1] for e in kept], dtype=np.complex128)
