"""Parameters of one sparse FFT run (readings of the paper's Theta(.) constants).

n, k      problem size and sparsity (Section 1 problem statement; n = 2^m per
          Section 2 Assumptions)
B, w      number of bins and window length (w a multiple of B)
alpha     flat-window transition fraction (Section 2 flat window definition)
delta     window accuracy (Section 2; the paper's 1/(4 n^2 L) is replaced by a
          fixed floating-point level)
theta     bin threshold; the paper's 1/2 for integer spectra (Algorithm 1) is a
          plan parameter here because coefficients need not be integers.  The
          default 1/4 (and g_min 0.4) avoid 1/2: with alpha = 1/2 and n/B a power
          of two, the offset o = C n is an integer where G' equals 1/2 up to
          rounding, which would make both tests exact ties.
g_min     smallest G'_{-o(i)} accepted when a bin value is divided by the window
b_min     exact mode: round r hashes into B_r = max(B >> r, b_min) bins with a
          window of w_r = w B_r / B samples (NoiselessSparseFFT of Algorithm 1
          shrinks the bin count with the remaining sparsity k_t = k / 2^t; alpha
          stays fixed, so w_r shrinks with B_r).  b_min = B keeps B fixed.
          General mode: a further floor on B_r (general.round_schedule).
patience  exact mode: stop after this many consecutive rounds with J empty.  One
          empty round is weak evidence: a remaining coefficient whose offset
          falls where G' is small is hidden in that round (the large-offset
          event of Section 3) with probability about alpha / 2.
stop_count  exact mode: also stop after `stop_patience` consecutive rounds with
          J empty once at least this many zhat entries exceed theta / 2 in
          magnitude (0: off).  With stop_count = k on an exactly k-sparse spectrum (the
          problem Algorithm 1 solves, with k known), k such entries and empty
          bins leave nothing to find unless a wrong entry stands in for a
          coefficient that stays invisible: one round is not enough, since a
          coefficient placed one location off and its residual can share a
          bin with equal window weight and cancel in the a = 0 hashing, and
          two can miss a small mislocated coefficient whose offsets fall in
          the transition band; below k entries the patience rule still
          applies.
stop_patience  empty rounds in a row that end a run under stop_count (>= 1).
ratio_tol  exact mode: decode only bins whose two hashings (shifts 0 and 1) agree
          in squared magnitude within this fraction (0: off).  An isolated
          coefficient gives equal magnitudes (the exact-estimation lemma of
          Section 3); a collision rarely does, and its decode would add a
          wrong entry that later rounds must take back out.
alpha_decay  exact mode: 0 (or 1) keeps alpha fixed; in (0, 1) round r uses
          alpha_r = alpha * alpha_decay^m, m = r up to the first round at the
          smallest bin count (alpha shrinking with B, as the alpha_t schedule
          of Section 3 does), with its window grown by 1 / alpha_decay^m
rounds    exact mode: maximum number of NoiselessSparseFFTInner rounds
          general mode: number of SparseFFT rounds
t, s      LocateInner region count and vote tolerance (Algorithm 3)
R_loc     LocateInner measurements per level (Algorithm 3)
R_est     EstimateValues measurements (Algorithm 2)
refine_shift  exact mode: 0 (off) or a third hashing per round at shift a = A
          (the multi-shift idea of LocateInner, Algorithm 3, used to estimate
          the phase with a few more samples): the pair's phase gives a coarse
          position p0, and the candidate c in [p0 - E, p0 + E] whose angle
          2 pi (A c mod n) / n is nearest the phase of u / u_A is taken
refine_window  E, the half-width of that candidate window
window    0: the Gaussian flat window of the Section 7 lemma; 1: the
          Kaiser-Bessel flat window (window.py kind 1), the same definition
          with about half the support
cap       largest output size (defaults to k)
literal   exact mode only: the paper-literal decode v = round(u_j) for integer
          spectra, without the bin and window checks
"""
import math
from dataclasses import dataclass


@dataclass
class SfftParams:
    n: int
    k: int
    B: int
    w: int
    seed: int
    alpha: float = 0.5
    delta: float = 1e-9
    theta: float = 0.25
    g_min: float = 0.4
    rounds: int = 8
    b_min: int = 0
    patience: int = 3
    stop_count: int = 0
    stop_patience: int = 2
    ratio_tol: float = 0.0
    alpha_decay: float = 0.0
    t: int = 16
    s: float = 0.125
    R_loc: int = 3
    R_est: int = 7
    refine_shift: int = 0
    refine_window: int = 16
    window: int = 0
    cap: int = 0
    literal: bool = False

    def _bins(self, r):
        floor = self.b_min if self.b_min > 0 else max(2, self.B >> 4)
        return max(self.B >> r, min(floor, self.B))

    def _decay_factor(self, r):
        """alpha_r / alpha: alpha_decay^m, m = r up to the first round at the
        smallest bin count (1 without decay)."""
        if not (0.0 < self.alpha_decay < 1.0):
            return 1.0
        r_floor = 0
        while r_floor + 1 < self.rounds and self._bins(r_floor + 1) != self._bins(r_floor):
            r_floor += 1
        return self.alpha_decay ** min(r, r_floor)

    def round_bins(self, r):
        """(B_r, w_r) of exact-mode round r.  With alpha_decay the window
        grows as alpha_r shrinks (sigma_g scales as B_r / alpha_r), rounded up
        to a multiple of B_r."""
        Br = self._bins(r)
        f = self._decay_factor(r)
        if f == 1.0:
            return Br, self.w * Br // self.B
        return Br, math.ceil((self.w // self.B) / f - 1e-9) * Br

    def round_alpha(self, r):
        """alpha_r of exact-mode round r (the alpha_t schedule of Section 3)."""
        return self.alpha * self._decay_factor(r)

    @property
    def out_cap(self):
        return self.cap if self.cap > 0 else self.k


def complex_median(vals):
    """Coordinate-wise median (separately in real and imaginary parts, as the
    comment of EstimateValues in Algorithm 2 says); an even count takes the
    mean of the two middle values."""
    import numpy as np

    v = np.asarray(vals, dtype=np.complex128)
    return complex(_median_real(v.real), _median_real(v.imag))


def _median_real(a):
    s = sorted(float(x) for x in a)
    m = len(s)
    if m % 2:
        return s[m // 2]
    return 0.5 * (s[m // 2 - 1] + s[m // 2])
