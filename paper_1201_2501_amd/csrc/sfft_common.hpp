// Shared host/device helpers of the sparse FFT library: counter draws,
// modular index arithmetic, the bin/offset map and the flat window G'.
//
// All index arithmetic is exact: n = 2^m divides 2^64, so uint64 products and
// sums that wrap modulo 2^64 are exact modulo n after masking with n - 1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define SFFT_HD __host__ __device__ __forceinline__

namespace sfft {

// ---------------------------------------------------------------- draws ----
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), the (c+1)-th output for a
// seed.  Every random choice of the method is one such draw; the counter
// layout is round<<32 | level<<20 | rep<<8 | purpose.
SFFT_HD uint64_t splitmix64(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

enum : uint32_t { PURPOSE_SIGMA = 1, PURPOSE_B = 2, PURPOSE_A = 3, PURPOSE_BETA = 4 };
constexpr uint32_t LEVEL_EST = 0xFFF;

SFFT_HD uint64_t draw_counter(uint64_t rnd, uint64_t level, uint64_t rep, uint64_t purpose) {
    return (rnd << 32) | (level << 20) | (rep << 8) | purpose;
}

SFFT_HD uint64_t draw(uint64_t seed, uint32_t rnd, uint32_t level, uint32_t rep, uint32_t purpose) {
    return splitmix64(seed, draw_counter(rnd, level, rep, purpose));
}

// sigma uniform among the odd residues mod n (n a power of two)
SFFT_HD uint64_t draw_sigma(uint64_t seed, uint64_t n, uint32_t rnd, uint32_t level = 0, uint32_t rep = 0) {
    return (draw(seed, rnd, level, rep, PURPOSE_SIGMA) & (n - 1)) | 1ull;
}
SFFT_HD uint64_t draw_b(uint64_t seed, uint64_t n, uint32_t rnd, uint32_t level = 0, uint32_t rep = 0) {
    return draw(seed, rnd, level, rep, PURPOSE_B) & (n - 1);
}
SFFT_HD uint64_t draw_a(uint64_t seed, uint64_t n, uint32_t rnd, uint32_t level, uint32_t rep) {
    return draw(seed, rnd, level, rep, PURPOSE_A) & (n - 1);
}
SFFT_HD uint64_t draw_beta(uint64_t seed, uint64_t lo, uint64_t hi, uint32_t rnd, uint32_t level, uint32_t rep) {
    return lo + draw(seed, rnd, level, rep, PURPOSE_BETA) % (hi - lo + 1ull);
}

// sigma^{-1} mod 2^64 for odd sigma by Newton-Hensel lifting: x = sigma is
// correct to 3 bits (sigma^2 = 1 mod 8), and x <- x (2 - sigma x) doubles the
// number of correct bits; five steps give 96 >= 64 bits.
SFFT_HD uint64_t inverse_odd(uint64_t sigma) {
    uint64_t x = sigma;
    for (int it = 0; it < 5; ++it) x *= 2ull - sigma * x;
    return x;
}

// ------------------------------------------------------------ bin map -----
// pi(i) = sigma (i - b) mod n; h = floor((pi B + n/2) / n) mod B (round half
// up); o = pi - h_unwrapped n / B in [-n/(2B), n/(2B)).  n and B are powers of
// two with B <= n and n B < 2^64, so both divisions are shifts.
struct BinOffset {
    uint32_t h;
    int64_t o;
};

SFFT_HD BinOffset bin_offset(uint64_t i, uint64_t sigma, uint64_t b, uint64_t n, uint64_t B) {
    const uint64_t mask = n - 1;
    const uint32_t ln = (uint32_t)__builtin_ctzll(n), lb = (uint32_t)__builtin_ctzll(B);
    const uint64_t pi = (sigma * ((i - b) & mask)) & mask;
    const uint64_t hu = ((pi << lb) + (n >> 1)) >> ln;
    BinOffset r;
    r.h = (uint32_t)(hu & (B - 1));
    r.o = (int64_t)pi - (int64_t)(hu << (ln - lb));
    return r;
}

// ------------------------------------------------------------ window G' ---
// G'_f of the flat window (Section 2 definition; Section 7 evaluation):
// 1 for |f| <= (1 - alpha) n / (2B), 0 for |f| >= n / (2B), otherwise
// Phi(sg (s + C)) - Phi(sg (s - C)) with s = |f| / n, evaluated as
// [erfc(sg (s - C)/sqrt 2) - erfc(sg (s + C)/sqrt 2)] / 2.  two_term = 0
// records that the second erfc is below 2^-60 of the first over the whole
// transition band, so subtracting it cannot change the FP64 result.
struct WindowShape {
    double sigma_g;
    double C;
    double alpha;
    uint32_t two_term;
    uint32_t pad;
    // Kaiser-Bessel window (plan field window = 1): G'_|f| for |f| <= n/(2B)
    // (device table, the window's response computed at plan time); nullptr
    // for the Gaussian window, whose G' has the closed form below
    const double* ftab;
};

SFFT_HD double gprime(int64_t f, uint64_t n, uint64_t B, WindowShape ws) {
    const uint64_t af = (uint64_t)(f < 0 ? -f : f);
    if ((double)(af * 2 * B) <= (1.0 - ws.alpha) * (double)n) return 1.0;
    if (af * 2 * B >= n) return 0.0;
    if (ws.ftab) return ws.ftab[af];
    const double s = (double)af / (double)n;
    const double r2 = 1.4142135623730951;
    const double lead = erfc(ws.sigma_g * (s - ws.C) / r2);
    return 0.5 * (ws.two_term ? lead - erfc(ws.sigma_g * (s + ws.C) / r2) : lead);
}

SFFT_HD int64_t floordiv(int64_t a, int64_t b) {   // b > 0
    int64_t q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

}  // namespace sfft
