"""Random draws of the method, from one counter-based generator.

The paper draws, per hashing, sigma uniform among the odd residues mod n and
shifts a, b uniform in [n] (Algorithm 1 NoiselessSparseFFTInner; Algorithm 2
EstimateValues; Algorithm 3 LocateSignal and LocateInner, which also draws the
integer beta from a range).  To reproduce a run from a seed, every draw is the
c-th output of SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) for that seed:

    z  = seed + (c + 1) * 0x9E3779B97F4A7C15            (mod 2^64)
    z  = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9           (mod 2^64)
    z  = (z ^ (z >> 27)) * 0x94D049BB133111EB           (mod 2^64)
    out = z ^ (z >> 31)

Counter layout: c = round << 32 | level << 20 | rep << 8 | purpose.
    exact mode   : (round r, level 0, rep 0)  -> sigma, b
    general mode : (round r, level 0, rep 0)  -> LocateSignal sigma, b
                   (round r, level D>=1, rep q) -> LocateInner a, beta
                   (round r, level EST, rep e) -> EstimateValues sigma, a, b
Reductions: sigma = (out mod n) | 1;  a, b = out mod n;
            beta = lo + out mod (hi - lo + 1).
"""

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15

PURPOSE_SIGMA = 1
PURPOSE_B = 2
PURPOSE_A = 3
PURPOSE_BETA = 4
LEVEL_EST = 0xFFF


def splitmix64(seed, c):
    z = (seed + (c + 1) * GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def counter(rnd, level, rep, purpose):
    return (rnd << 32) | (level << 20) | (rep << 8) | purpose


def draw(seed, rnd, level, rep, purpose):
    return splitmix64(seed & MASK64, counter(rnd, level, rep, purpose))


def draw_sigma(seed, n, rnd, level=0, rep=0):
    """sigma uniform among odd residues mod n."""
    return (draw(seed, rnd, level, rep, PURPOSE_SIGMA) % n) | 1


def draw_b(seed, n, rnd, level=0, rep=0):
    return draw(seed, rnd, level, rep, PURPOSE_B) % n


def draw_a(seed, n, rnd, level, rep):
    return draw(seed, rnd, level, rep, PURPOSE_A) % n


def draw_beta(seed, lo, hi, rnd, level, rep):
    return lo + draw(seed, rnd, level, rep, PURPOSE_BETA) % (hi - lo + 1)


def inverse_mod(sigma, n):
    """sigma^{-1} mod n for odd sigma (extended Euclid via Python's pow)."""
    return pow(int(sigma), -1, int(n))
