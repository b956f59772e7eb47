// HIP kernels of the sparse FFT hot path for gfx950 (CDNA4, wave64).
//
//  * k_h2b_pair      HashToBins at two shifts (a, a + beta) of one permutation
//                    (sigma, b): permuted gather, window x modulation, fold
//                    into B residues, B-point FFT in LDS, * sqrt(n).  One
//                    workgroup per (signal, round).  The gather is HBM bound:
//                    every sample is an independent 8- or 16-byte read at
//                    sigma (t - a) mod n, accumulated in registers by the
//                    thread that owns its residue t mod B (no atomics, fixed
//                    summation order).
//  * k_h2b_split     the same accumulation split over many workgroups by
//                    window range (one signal at a time), partial sums to HBM
//  * k_h2b_reduce    fixed-order sum of the partials, modulation, FFT
//  * k_exact_*       exact-mode decode (Algorithm 1): subtract zhat in the
//                    bins, threshold, phase decode, bin check, merge into the
//                    sorted zhat; then the FP64 median re-estimation and output.
#include "sfft_internal.hpp"

namespace sfft {

template <class T>
struct cx {
    T r, i;
};

template <class T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <class T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <class T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <class T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.r * s, a.i * s}; }

template <class T>
__device__ __forceinline__ cx<T> to_cx(cx<double> a) { return {(T)a.r, (T)a.i}; }

// omega^p = exp(-2 pi i p / n) from the exact integer p in [0, n), in FP64.
__device__ __forceinline__ cx<double> omega_d(uint64_t p, uint64_t n) {
    double s, c;
    sincospi(2.0 * (double)p / (double)n, &s, &c);
    return {c, -s};
}

__device__ __forceinline__ uint32_t bitrev(uint32_t j, uint32_t logB) {
    return logB ? (__brev(j) >> (32 - logB)) : 0u;
}

template <class T>
struct TwTraits;
template <>
struct TwTraits<double> {
    using V = double2;
};
template <>
struct TwTraits<float> {
    using V = float2;
};

// In-place radix-2 decimation-in-frequency FFT of VA and VB (B points each,
// natural-order input, bit-reversed output), unnormalised, sign -:
// X_j = sum_r V_r exp(-2 pi i j r / B).  tw holds exp(-2 pi i m / Bmax),
// m < Bmax.
template <class TA>
__device__ void lds_fft2(cx<TA>* VA, cx<TA>* VB, uint32_t B, uint32_t Bmax,
                         const typename TwTraits<TA>::V* tw) {
    const uint32_t tid = threadIdx.x;
    const uint32_t hb = B >> 1;
    for (uint32_t half = hb; half >= 1; half >>= 1) {
        const uint32_t tstride = Bmax / (2 * half);
        for (uint32_t k = tid; k < B; k += kThreads) {
            cx<TA>* V = k < hb ? VA : VB;
            const uint32_t kk = k & (hb - 1);
            const uint32_t j = kk & (half - 1);
            const uint32_t i0 = ((kk - j) << 1) + j;
            const uint32_t i1 = i0 + half;
            const cx<TA> a = V[i0], b = V[i1];
            const auto t = tw[j * tstride];
            V[i0] = cadd(a, b);
            V[i1] = cmul(csub(a, b), cx<TA>{t.x, t.y});
        }
        __syncthreads();
    }
}

// Accumulate one hashing pair over the samples t_A in [seg_lo, seg_hi) whose
// window index L = (t_A - r) / B lies in [Lwin_lo, Lwin_hi].  Sample t_A is
// x[sigma (t_A - a)]; it enters hashing A at t = t_A with weight G_{t_A} and
// hashing B (shift a + beta) at t = t_A + beta with weight G_{t_A + beta}.
// The modulation omega^{c t}, c = sigma b, is split as omega^{c r} (applied
// per residue later) times M_L = omega^{c B L} (table in LDS).  Partial sums
// are added into VA/VB[part * B + r].
template <class TIn, class TA>
__device__ void accumulate_pair(const TIn* __restrict__ x, const TA* __restrict__ G, cx<TA>* VA,
                                cx<TA>* VB, cx<TA>* M, uint64_t n, uint64_t sigma, uint64_t a,
                                uint64_t beta, uint64_t b, uint32_t B, uint32_t logB, uint64_t w,
                                int64_t t0, int64_t Lwin_lo, int64_t Lwin_hi, uint32_t parts) {
    const uint32_t tid = threadIdx.x;
    const uint64_t mask = n - 1;
    const uint64_t c = (sigma * b) & mask;
    const uint64_t cB = (c * (uint64_t)B) & mask;
    const uint64_t sB = (sigma * (uint64_t)B) & mask;
    const int64_t iB = (int64_t)B;
    const int64_t iw = (int64_t)w;
    const int64_t ibeta = (int64_t)beta;
    int64_t lo[2], hi[2];
    int nseg;
    if (beta < w) {
        lo[0] = t0 - ibeta;
        hi[0] = t0 + iw;
        nseg = 1;
    } else {
        lo[0] = t0 - ibeta;
        hi[0] = lo[0] + iw;
        lo[1] = t0;
        hi[1] = t0 + iw;
        nseg = 2;
    }
    for (int sg = 0; sg < nseg; ++sg) {
        int64_t Llo = floordiv(lo[sg] - (iB - 1), iB);
        int64_t Lhi = floordiv(hi[sg] - 1, iB);
        Llo = Llo > Lwin_lo ? Llo : Lwin_lo;
        Lhi = Lhi < Lwin_hi ? Lhi : Lwin_hi;
        if (Llo > Lhi) continue;   // uniform over the block
        __syncthreads();
        for (int64_t L = Llo + tid; L <= Lhi; L += kThreads)
            M[L - Llo] = to_cx<TA>(omega_d((cB * (uint64_t)L) & mask, n));
        __syncthreads();
        for (uint32_t slot = tid; slot < parts * B; slot += kThreads) {
            const uint32_t part = slot >> logB;
            const uint32_t r = slot & (B - 1);
            int64_t L0 = floordiv(lo[sg] - (int64_t)r + iB - 1, iB);
            int64_t L1 = floordiv(hi[sg] - 1 - (int64_t)r, iB);
            L0 = L0 > Llo ? L0 : Llo;
            L1 = L1 < Lhi ? L1 : Lhi;
            if (parts > 1) {
                const int64_t len = L1 - L0 + 1;
                if (len <= 0) continue;
                const int64_t chunk = (len + parts - 1) / parts;
                const int64_t b0 = L0 + (int64_t)part * chunk;
                const int64_t b1 = b0 + chunk - 1;
                L0 = b0;
                L1 = b1 < L1 ? b1 : L1;
            }
            if (L0 > L1) continue;
            int64_t tA = (int64_t)r + L0 * iB;
            uint64_t idx = ((uint64_t)(tA - (int64_t)a) * sigma) & mask;
            TA aAr = 0, aAi = 0, aBr = 0, aBi = 0;
            const cx<TA>* Mp = M + (L0 - Llo);
            const int64_t cnt = L1 - L0 + 1;
#pragma unroll 4
            for (int64_t q = 0; q < cnt; ++q) {
                const TIn xv = x[idx];
                const int64_t uA = tA - t0;
                const int64_t uB = uA + ibeta;
                const bool inA = (uA >= 0) & (uA < iw);
                const bool inB = (uB >= 0) & (uB < iw);
                const TA gA = inA ? G[inA ? uA : 0] : (TA)0;
                const TA gB = inB ? G[inB ? uB : 0] : (TA)0;
                const cx<TA> m = Mp[q];
                const TA xr = (TA)xv.x, xi = (TA)xv.y;
                const TA pr = m.r * xr - m.i * xi;
                const TA pi = m.r * xi + m.i * xr;
                aAr += gA * pr;
                aAi += gA * pi;
                aBr += gB * pr;
                aBi += gB * pi;
                idx = (idx + sB) & mask;
                tA += iB;
            }
            VA[slot] = cadd(VA[slot], cx<TA>{aAr, aAi});
            VB[slot] = cadd(VB[slot], cx<TA>{aBr, aBi});
        }
    }
}

// Sum the parts of column r, apply omega^{c r} (hashing A) and
// omega^{c (r + beta)} (hashing B), leaving natural-order folds in VA/VB[0, B).
template <class TA>
__device__ void finalize_folds(cx<TA>* VA, cx<TA>* VB, uint64_t n, uint64_t sigma, uint64_t b,
                               uint64_t beta, uint32_t B, uint32_t parts) {
    const uint64_t mask = n - 1;
    const uint64_t c = (sigma * b) & mask;
    for (uint32_t r = threadIdx.x; r < B; r += kThreads) {
        cx<TA> sa = VA[r], sb = VB[r];
        for (uint32_t p = 1; p < parts; ++p) {
            sa = cadd(sa, VA[p * B + r]);
            sb = cadd(sb, VB[p * B + r]);
        }
        const cx<TA> baseA = to_cx<TA>(omega_d((c * (uint64_t)r) & mask, n));
        const cx<TA> baseB = to_cx<TA>(omega_d((c * ((uint64_t)r + beta)) & mask, n));
        VA[r] = cmul(baseA, sa);
        VB[r] = cmul(baseB, sb);
    }
}

// After lds_fft2: bin j of A is VA[bitrev j]; hashing B was folded by the
// residue of t_A, so its bin j carries the extra factor exp(-2 pi i j beta / B).
template <class TA>
__device__ void store_bins(const cx<TA>* VA, const cx<TA>* VB, uint32_t B, uint32_t logB, uint32_t Bmax,
                           uint64_t beta, const typename TwTraits<TA>::V* tw, double sqrt_n,
                           double* out0, double* out1) {
    const uint32_t bstride = Bmax / B;
    for (uint32_t j = threadIdx.x; j < B; j += kThreads) {
        const uint32_t br = bitrev(j, logB);
        const cx<TA> va = VA[br];
        cx<TA> vb = VB[br];
        const uint32_t e = (uint32_t)(((uint64_t)j * (beta & (B - 1))) & (B - 1));
        const auto t = tw[e * bstride];
        vb = cmul(vb, cx<TA>{t.x, t.y});
        out0[2 * j] = (double)va.r * sqrt_n;
        out0[2 * j + 1] = (double)va.i * sqrt_n;
        out1[2 * j] = (double)vb.r * sqrt_n;
        out1[2 * j + 1] = (double)vb.i * sqrt_n;
    }
}

template <class TIn, class TA>
__global__ void __launch_bounds__(kThreads) k_h2b_pair(H2BArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t sig, r, ro;
    const uint64_t n = A.n;
    uint64_t sigma, a, beta, b;
    if (A.explicit_job) {
        sig = 0;
        r = A.round_lo;
        ro = 0;
        sigma = A.sigma;
        a = A.a;
        beta = A.beta;
        b = A.b;
    } else if (A.jobs) {
        // general mode: LocateInner pair (level, rep) or EstimateValues hashing
        const uint32_t job = blockIdx.x / A.count;
        sig = blockIdx.x - job * A.count;
        const GenJob jb = A.jobs[job];
        r = jb.round;
        ro = jb.slot;
        const uint64_t seed = A.seeds ? A.seeds[sig] : A.plan_seed;
        const GenRoundDev& gr = A.groundv[r];
        if (jb.index < gr.nloc) {
            const uint32_t D = jb.index / A.R_loc + 1, q = jb.index % A.R_loc;
            sigma = draw_sigma(seed, n, r, 0, 0);
            b = draw_b(seed, n, r, 0, 0);
            a = draw_a(seed, n, r, D, q);
            beta = draw_beta(seed, gr.blo[D - 1], gr.bhi[D - 1], r, D, q);
        } else {
            const uint32_t e = jb.index - gr.nloc;
            sigma = draw_sigma(seed, n, r, LEVEL_EST, e);
            a = draw_a(seed, n, r, LEVEL_EST, e);
            b = draw_b(seed, n, r, LEVEL_EST, e);
            beta = 0;
        }
    } else {
        const uint32_t rr = blockIdx.x / A.count;
        sig = blockIdx.x - rr * A.count;
        r = A.round_lo + rr;
        ro = r;
        const uint64_t seed = A.seeds ? A.seeds[sig] : A.plan_seed;
        sigma = draw_sigma(seed, n, r);
        b = draw_b(seed, n, r);
        a = 0;
        beta = 1;
    }
    const RoundDev g = A.geom[r];
    const TIn* x = reinterpret_cast<const TIn*>(A.x) + (uint64_t)sig * A.sig_stride;
    const TA* G = reinterpret_cast<const TA*>(A.gtab) + g.gofs;
    const auto* tw = reinterpret_cast<const typename TwTraits<TA>::V*>(A.tw);
    const uint32_t B = g.B;
    const uint32_t parts = B >= kThreads ? 1u : kThreads / B;
    cx<TA>* VA = reinterpret_cast<cx<TA>*>(smem);
    cx<TA>* VB = VA + parts * B;
    cx<TA>* M = VB + parts * B;
    for (uint32_t q = threadIdx.x; q < parts * B; q += kThreads) {
        VA[q] = cx<TA>{0, 0};
        VB[q] = cx<TA>{0, 0};
    }
    accumulate_pair<TIn, TA>(x, G, VA, VB, M, n, sigma, a, beta, b, B, g.logB, g.w, g.t0,
                             INT64_MIN / 4, INT64_MAX / 4, parts);
    __syncthreads();
    finalize_folds<TA>(VA, VB, n, sigma, b, beta, B, parts);
    __syncthreads();
    lds_fft2<TA>(VA, VB, B, A.Bmax, tw);
    double* out0 = A.raw + (((uint64_t)sig * A.raw_rounds + ro) * 2) * (uint64_t)A.Bmax * 2;
    store_bins<TA>(VA, VB, B, g.logB, A.Bmax, beta, tw, A.sqrt_n, out0, out0 + 2 * (uint64_t)A.Bmax);
}

// Plain path, stage 1: block p accumulates window chunk p (lchunk values of L)
// of round `round`, signal 0, and writes unmodulated partial folds.
template <class TIn, class TA>
__global__ void __launch_bounds__(kThreads) k_h2b_split(H2BArgs A, uint32_t round) {
    extern __shared__ __align__(16) unsigned char smem[];
    const RoundDev g = A.geom[round];
    const uint64_t n = A.n;
    const uint64_t sigma = A.sigma, a = A.a, beta = A.beta, b = A.b;
    const TIn* x = reinterpret_cast<const TIn*>(A.x);
    const TA* G = reinterpret_cast<const TA*>(A.gtab) + g.gofs;
    const uint32_t B = g.B;
    const uint32_t parts = B >= kThreads ? 1u : kThreads / B;
    cx<TA>* VA = reinterpret_cast<cx<TA>*>(smem);
    cx<TA>* VB = VA + parts * B;
    cx<TA>* M = VB + parts * B;
    for (uint32_t q = threadIdx.x; q < parts * B; q += kThreads) {
        VA[q] = cx<TA>{0, 0};
        VB[q] = cx<TA>{0, 0};
    }
    const int64_t iB = (int64_t)B;
    const int64_t Lmin = floordiv(g.t0 - (int64_t)beta - (iB - 1), iB);
    const int64_t Llo = Lmin + (int64_t)blockIdx.x * A.lchunk;
    const int64_t Lhi = Llo + A.lchunk - 1;
    accumulate_pair<TIn, TA>(x, G, VA, VB, M, n, sigma, a, beta, b, B, g.logB, g.w, g.t0, Llo, Lhi, parts);
    __syncthreads();
    double* out = A.partial + (uint64_t)blockIdx.x * 4 * B;
    for (uint32_t r = threadIdx.x; r < B; r += kThreads) {
        cx<TA> sa = VA[r], sb = VB[r];
        for (uint32_t p = 1; p < parts; ++p) {
            sa = cadd(sa, VA[p * B + r]);
            sb = cadd(sb, VB[p * B + r]);
        }
        out[2 * r] = (double)sa.r;
        out[2 * r + 1] = (double)sa.i;
        out[2 * B + 2 * r] = (double)sb.r;
        out[2 * B + 2 * r + 1] = (double)sb.i;
    }
}

// Plain path, stage 2: one block sums the partials in part order, applies the
// modulation, runs the FFT and stores the bins of round `round` (signal 0).
template <class TA>
__global__ void __launch_bounds__(kThreads) k_h2b_reduce(H2BArgs A, uint32_t round) {
    extern __shared__ __align__(16) unsigned char smem[];
    const RoundDev g = A.geom[round];
    const uint32_t B = g.B;
    cx<TA>* VA = reinterpret_cast<cx<TA>*>(smem);
    cx<TA>* VB = VA + B;
    const auto* tw = reinterpret_cast<const typename TwTraits<TA>::V*>(A.tw);
    for (uint32_t r = threadIdx.x; r < B; r += kThreads) {
        double ar = 0, ai = 0, br = 0, bi = 0;
        for (uint32_t p = 0; p < A.parts; ++p) {
            const double* q = A.partial + (uint64_t)p * 4 * B;
            ar += q[2 * r];
            ai += q[2 * r + 1];
            br += q[2 * B + 2 * r];
            bi += q[2 * B + 2 * r + 1];
        }
        VA[r] = cx<TA>{(TA)ar, (TA)ai};
        VB[r] = cx<TA>{(TA)br, (TA)bi};
    }
    __syncthreads();
    finalize_folds<TA>(VA, VB, A.n, A.sigma, A.b, A.beta, B, 1);
    __syncthreads();
    lds_fft2<TA>(VA, VB, B, A.Bmax, tw);
    double* out0 = A.raw + ((uint64_t)round * 2) * (uint64_t)A.Bmax * 2;
    store_bins<TA>(VA, VB, B, g.logB, A.Bmax, A.beta, tw, A.sqrt_n, out0, out0 + 2 * (uint64_t)A.Bmax);
}

// ------------------------------------------------------------------------
// Block-wide helpers for the decode kernels.

// Bitonic sort (ascending) of N = power-of-two 64-bit keys in LDS.
__device__ void bitonic_sort_u64(uint64_t* key, uint32_t N) {
    for (uint32_t size = 2; size <= N; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (uint32_t t = threadIdx.x; t < N / 2; t += kThreads) {
                const uint32_t lo = 2 * t - (t & (stride - 1));
                const uint32_t hi = lo + stride;
                const bool up = ((lo & size) == 0);
                const uint64_t a = key[lo], b = key[hi];
                if ((a > b) == up) {
                    key[lo] = b;
                    key[hi] = a;
                }
            }
        }
    }
    __syncthreads();
}

__device__ __forceinline__ uint32_t pow2_at_least(uint32_t v) {
    uint32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Exclusive prefix sum of one value per thread; returns the block total.
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* scratch, uint32_t* out_prefix) {
    const uint32_t tid = threadIdx.x;
    __syncthreads();
    scratch[tid] = v;
    __syncthreads();
    for (uint32_t off = 1; off < kThreads; off <<= 1) {
        const uint32_t add = tid >= off ? scratch[tid - off] : 0u;
        __syncthreads();
        scratch[tid] += add;
        __syncthreads();
    }
    *out_prefix = scratch[tid] - v;
    const uint32_t total = scratch[kThreads - 1];
    __syncthreads();
    return total;
}

constexpr uint32_t kKeyBinShift = 20;                 // zhat sort key: bin << 20 | entry
constexpr uint64_t kEntryMask = (1ull << kKeyBinShift) - 1;
constexpr uint32_t kCandShift = 13;                   // candidate key: i << 13 | bin
constexpr uint64_t kNone = ~0ull;

struct DecodeShared {
    uint64_t key[kMaxZ];       // sort space (64 KiB)
    uint32_t scan[kThreads];
    uint32_t nJ;
    uint32_t flag;
};

__device__ __forceinline__ const double* raw_bins(const DecodeArgs& D, uint32_t sig, uint32_t r, uint32_t a) {
    return D.raw + (((uint64_t)sig * D.rounds + r) * 2 + a) * (uint64_t)D.Bmax * 2;
}

// lower_bound over a sorted uint64 array in global memory
__device__ __forceinline__ uint32_t lower_bound_g(const uint64_t* arr, uint32_t len, uint64_t v) {
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (arr[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Sort zhat entries e < zc by (bin of round geometry, e) into S.key.
__device__ void sort_entries_by_bin(DecodeShared& S, const uint64_t* zi, uint32_t zc, uint64_t sigma,
                                    uint64_t b, uint64_t n, uint32_t B) {
    const uint32_t N = pow2_at_least(zc);
    for (uint32_t e = threadIdx.x; e < N; e += kThreads) {
        if (e < zc) {
            const BinOffset bo = bin_offset(zi[e], sigma, b, n, B);
            S.key[e] = ((uint64_t)bo.h << kKeyBinShift) | e;
        } else {
            S.key[e] = kNone;
        }
    }
    bitonic_sort_u64(S.key, N);
}

// zhat += candidates.  S.key[0, NB) holds candidate keys i << 13 | slot
// (kNone for empty slots), sorted ascending; cv[slot] is the value.  Existing
// indices are updated in place, new ones are merged (by index) into the other
// zhat buffer, which becomes current.  Returns the number of new entries.
__device__ uint32_t merge_candidates(DecodeShared& S, uint32_t NB, const double* cv, uint64_t* zidx_all,
                                     double* zval_all, uint32_t sig, uint32_t capz, uint32_t* st) {
    const uint32_t tid = threadIdx.x;
    const uint32_t zc = st[ST_ZCOUNT];
    const uint32_t zb = st[ST_ZBUF];
    uint64_t* zi = zidx_all + ((uint64_t)sig * 2 + zb) * capz;
    double* zv = zval_all + ((uint64_t)sig * 2 + zb) * capz * 2;
    const uint64_t slot_mask = (1ull << kCandShift) - 1;
    for (uint32_t q = tid; q < NB; q += kThreads) {
        const uint64_t k = S.key[q];
        if (k == kNone) continue;
        const uint64_t i = k >> kCandShift;
        const uint32_t j = (uint32_t)(k & slot_mask);
        const uint32_t e = lower_bound_g(zi, zc, i);
        if (e < zc && zi[e] == i) {
            zv[2 * e] += cv[2 * j];
            zv[2 * e + 1] += cv[2 * j + 1];
            S.key[q] = kNone;
        }
    }
    __syncthreads();
    bitonic_sort_u64(S.key, NB);   // new entries first, ascending index
    uint32_t mycnt = 0;
    for (uint32_t q = tid; q < NB; q += kThreads) mycnt += S.key[q] != kNone;
    if (tid == 0) S.flag = 0;
    __syncthreads();
    if (mycnt) atomicAdd(&S.flag, mycnt);
    __syncthreads();
    uint32_t mnew = S.flag;
    if (zc + mnew > capz) {
        mnew = capz - zc;
        if (tid == 0) st[ST_FLAGS] |= 2u;
    }
    uint64_t* zo = zidx_all + ((uint64_t)sig * 2 + (zb ^ 1)) * capz;
    double* zov = zval_all + ((uint64_t)sig * 2 + (zb ^ 1)) * capz * 2;
    for (uint32_t e = tid; e < zc; e += kThreads) {
        const uint64_t i = zi[e];
        uint32_t lo = 0, hi = mnew;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if ((S.key[mid] >> kCandShift) < i) lo = mid + 1; else hi = mid;
        }
        const uint32_t pos = e + lo;
        zo[pos] = i;
        zov[2 * pos] = zv[2 * e];
        zov[2 * pos + 1] = zv[2 * e + 1];
    }
    for (uint32_t q = tid; q < mnew; q += kThreads) {
        const uint64_t i = S.key[q] >> kCandShift;
        const uint32_t j = (uint32_t)(S.key[q] & slot_mask);
        const uint32_t pos = q + lower_bound_g(zi, zc, i);
        zo[pos] = i;
        zov[2 * pos] = cv[2 * j];
        zov[2 * pos + 1] = cv[2 * j + 1];
    }
    __syncthreads();
    if (tid == 0) {
        st[ST_ZCOUNT] = zc + mnew;
        st[ST_ZBUF] = zb ^ 1;
    }
    __syncthreads();
    return mnew;
}

// One round of NoiselessSparseFFTInner on signal `sig` (Algorithm 1).
__device__ void exact_round(const DecodeArgs& D, DecodeShared& S, uint32_t sig, uint32_t r, uint64_t seed) {
    const uint32_t tid = threadIdx.x;
    const RoundDev g = D.geom[r];
    const uint64_t n = D.n, mask = n - 1;
    const uint32_t B = g.B;
    const uint64_t sigma = draw_sigma(seed, n, r);
    const uint64_t b = draw_b(seed, n, r);
    const uint64_t sinv = inverse_odd(sigma) & mask;
    uint32_t* st = D.state + (uint64_t)sig * kStateWords;
    const uint32_t zc = st[ST_ZCOUNT];
    const uint32_t zb = st[ST_ZBUF];
    uint64_t* zi = D.zidx + ((uint64_t)sig * 2 + zb) * D.capz;
    double* zv = D.zval + ((uint64_t)sig * 2 + zb) * D.capz * 2;
    double* w0 = D.work + (uint64_t)sig * 4 * D.Bmax;
    double* w1 = w0 + 2 * (uint64_t)D.Bmax;
    const double* r0 = raw_bins(D, sig, r, 0);
    const double* r1 = raw_bins(D, sig, r, 1);
    for (uint32_t j = tid; j < 2 * B; j += kThreads) {
        w0[j] = r0[j];
        w1[j] = r1[j];
    }
    // HashToBins step 4: u_{h(i)} -= G'_{-o(i)} zhat_i omega^{a sigma i}, per bin
    // in ascending index order.
    if (zc > 0) {
        sort_entries_by_bin(S, zi, zc, sigma, b, n, B);
        for (uint32_t p = tid; p < zc; p += kThreads) {
            const uint64_t h = S.key[p] >> kKeyBinShift;
            if (p > 0 && (S.key[p - 1] >> kKeyBinShift) == h) continue;
            double u0r = w0[2 * h], u0i = w0[2 * h + 1];
            double u1r = w1[2 * h], u1i = w1[2 * h + 1];
            for (uint32_t q = p; q < zc && (S.key[q] >> kKeyBinShift) == h; ++q) {
                const uint32_t e = (uint32_t)(S.key[q] & kEntryMask);
                const uint64_t i = zi[e];
                const BinOffset bo = bin_offset(i, sigma, b, n, B);
                const double gp = gprime(-bo.o, n, B, g.ws);
                const double c0r = gp * zv[2 * e], c0i = gp * zv[2 * e + 1];
                const cx<double> om = omega_d((sigma * i) & mask, n);
                const cx<double> c1 = cmul(cx<double>{c0r, c0i}, om);
                u0r -= c0r;
                u0i -= c0i;
                u1r -= c1.r;
                u1i -= c1.i;
            }
            w0[2 * h] = u0r;
            w0[2 * h + 1] = u0i;
            w1[2 * h] = u1r;
            w1[2 * h + 1] = u1i;
        }
    }
    if (tid == 0) S.nJ = 0;
    __syncthreads();
    // threshold, phase decode, bin and window checks
    uint32_t myJ = 0;
    const double two_pi = 6.283185307179586;
    for (uint32_t j = tid; j < B; j += kThreads) {
        const double u0r = w0[2 * j], u0i = w0[2 * j + 1];
        const double mag = sqrt(u0r * u0r + u0i * u0i);
        uint64_t ci = kNone;
        if (mag > D.theta) {
            ++myJ;
            const double u1r = w1[2 * j], u1i = w1[2 * j + 1];
            const double zr = u0r * u1r + u0i * u1i;
            const double zim = u0i * u1r - u0r * u1i;
            double phi = atan2(zim, zr);
            if (phi < 0.0) phi += two_pi;
            const double q = phi / two_pi * (double)n;
            const uint64_t pos = ((uint64_t)floor(q + 0.5)) & mask;
            const uint64_t i = (sinv * pos) & mask;
            const BinOffset bo = bin_offset(i, sigma, b, n, B);
            if (bo.h == j) {
                const double gp = gprime(-bo.o, n, B, g.ws);
                if (gp >= D.g_min) {
                    ci = i;
                    D.cand_v[((uint64_t)sig * D.Bmax + j) * 2] = u0r / gp;
                    D.cand_v[((uint64_t)sig * D.Bmax + j) * 2 + 1] = u0i / gp;
                }
            }
        }
        D.cand_i[(uint64_t)sig * D.Bmax + j] = ci;
    }
    if (myJ) atomicAdd(&S.nJ, myJ);
    __syncthreads();
    const uint32_t J = S.nJ;
    if (J == 0) {
        if (tid == 0) {
            st[ST_EMPTY] += 1;
            if (st[ST_EMPTY] >= D.patience) st[ST_DONE] = 1;
            st[ST_ROUNDS] = r + 1;
            st[ST_LASTJ] = 0;
            st[ST_ACCEPT] = 0;
        }
        __syncthreads();
        return;
    }
    // candidates sorted by index: key = i << 13 | j
    const uint32_t NB = pow2_at_least(B);
    const uint64_t* ci_arr = D.cand_i + (uint64_t)sig * D.Bmax;
    const double* cv_arr = D.cand_v + (uint64_t)sig * D.Bmax * 2;
    for (uint32_t j = tid; j < NB; j += kThreads) {
        const uint64_t ci = j < B ? ci_arr[j] : kNone;
        S.key[j] = ci == kNone ? kNone : ((ci << kCandShift) | j);
    }
    bitonic_sort_u64(S.key, NB);
    const uint32_t mnew = merge_candidates(S, NB, cv_arr, D.zidx, D.zval, sig, D.capz, st);
    if (tid == 0) {
        st[ST_EMPTY] = 0;
        st[ST_ROUNDS] = r + 1;
        st[ST_LASTJ] = J;
        st[ST_ACCEPT] = mnew;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kThreads) k_exact_init(DecodeArgs D) {
    const uint32_t sig = blockIdx.x * kThreads + threadIdx.x;
    if (sig >= D.count) return;
    uint32_t* st = D.state + (uint64_t)sig * kStateWords;
    for (uint32_t q = 0; q < kStateWords; ++q) st[q] = 0;
}

__global__ void __launch_bounds__(kThreads) k_exact_decode(DecodeArgs D) {
    __shared__ DecodeShared S;
    const uint32_t sig = blockIdx.x;
    const uint64_t seed = D.seeds ? D.seeds[sig] : D.plan_seed;
    const uint32_t* st = D.state + (uint64_t)sig * kStateWords;
    for (uint32_t r = D.r_begin; r < D.r_end; ++r) {
        __syncthreads();
        if (st[ST_DONE]) break;
        exact_round(D, S, sig, r, seed);
    }
}

// Final FP64 re-estimation (median over the decoded rounds of the bin value
// with the other recovered coefficients removed, divided by G') and output.
__global__ void __launch_bounds__(kThreads) k_exact_finish(DecodeArgs D) {
    __shared__ DecodeShared S;
    const uint32_t tid = threadIdx.x;
    const uint32_t sig = blockIdx.x;
    const uint64_t seed = D.seeds ? D.seeds[sig] : D.plan_seed;
    uint32_t* st = D.state + (uint64_t)sig * kStateWords;
    const uint64_t n = D.n, mask = n - 1;
    const uint32_t zc = st[ST_ZCOUNT];
    const uint32_t zb = st[ST_ZBUF];
    const uint32_t R = st[ST_ROUNDS];
    const uint64_t* zi = D.zidx + ((uint64_t)sig * 2 + zb) * D.capz;
    const double* zv = D.zval + ((uint64_t)sig * 2 + zb) * D.capz * 2;
    double* est = D.est + (uint64_t)sig * D.capz * D.rounds * 2;
    uint32_t* ecount = D.ecount + (uint64_t)sig * D.capz;
    double* gtmp = D.gtmp + (uint64_t)sig * D.capz;
    for (uint32_t e = tid; e < zc; e += kThreads) ecount[e] = 0;
    for (uint32_t r = 0; r < R; ++r) {
        const RoundDev g = D.geom[r];
        const uint32_t B = g.B;
        const uint64_t sigma = draw_sigma(seed, n, r);
        const uint64_t b = draw_b(seed, n, r);
        __syncthreads();
        for (uint32_t e = tid; e < zc; e += kThreads) {
            const BinOffset bo = bin_offset(zi[e], sigma, b, n, B);
            gtmp[e] = gprime(-bo.o, n, B, g.ws);
        }
        sort_entries_by_bin(S, zi, zc, sigma, b, n, B);
        const double* r0 = raw_bins(D, sig, r, 0);
        for (uint32_t p = tid; p < zc; p += kThreads) {
            const uint32_t e = (uint32_t)(S.key[p] & kEntryMask);
            const double ge = gtmp[e];
            if (ge < D.g_min) continue;
            const uint64_t h = S.key[p] >> kKeyBinShift;
            uint32_t s0 = p;
            while (s0 > 0 && (S.key[s0 - 1] >> kKeyBinShift) == h) --s0;
            double orr = 0.0, oii = 0.0;
            uint32_t members = 0;
            for (uint32_t q = s0; q < zc && (S.key[q] >> kKeyBinShift) == h; ++q) {
                ++members;
                const uint32_t e2 = (uint32_t)(S.key[q] & kEntryMask);
                if (e2 == e) continue;
                orr += gtmp[e2] * zv[2 * e2];
                oii += gtmp[e2] * zv[2 * e2 + 1];
            }
            // samples of rounds where e is alone in its bin fill the count from
            // the front, the others from the back of the entry's slot range
            const uint32_t c = ecount[e];
            const uint32_t na = c & 0xFFFFu, nb = c >> 16;
            const uint32_t slot = members == 1 ? na : D.rounds - 1 - nb;
            est[((uint64_t)e * D.rounds + slot) * 2] = (r0[2 * h] - orr) / ge;
            est[((uint64_t)e * D.rounds + slot) * 2 + 1] = (r0[2 * h + 1] - oii) / ge;
            ecount[e] = members == 1 ? c + 1 : c + (1u << 16);
        }
    }
    __syncthreads();
    // medians into the est slot 0 (re, im); survivors |v| > theta / 2
    uint32_t mysurv = 0;
    const double half_theta = 0.5 * D.theta;
    double* fin = D.fin + (uint64_t)sig * D.capz * 2;
    for (uint32_t e = tid; e < zc; e += kThreads) {
        // median over the rounds where e was alone in its bin, else over all
        const uint32_t na = ecount[e] & 0xFFFFu, nb = ecount[e] >> 16;
        const uint32_t c = na ? na : nb;
        const uint32_t first = na ? 0u : D.rounds - nb;
        double vr = zv[2 * e], vi = zv[2 * e + 1];
        if (c > 0) {
            double re[kMaxRounds], im[kMaxRounds];
            for (uint32_t q = 0; q < c; ++q) {
                re[q] = est[((uint64_t)e * D.rounds + first + q) * 2];
                im[q] = est[((uint64_t)e * D.rounds + first + q) * 2 + 1];
            }
            for (uint32_t q = 1; q < c; ++q) {
                const double a = re[q], bq = im[q];
                int32_t s = (int32_t)q - 1;
                while (s >= 0 && re[s] > a) { re[s + 1] = re[s]; --s; }
                re[s + 1] = a;
                s = (int32_t)q - 1;
                while (s >= 0 && im[s] > bq) { im[s + 1] = im[s]; --s; }
                im[s + 1] = bq;
            }
            if (c & 1) {
                vr = re[c / 2];
                vi = im[c / 2];
            } else {
                vr = 0.5 * (re[c / 2 - 1] + re[c / 2]);
                vi = 0.5 * (im[c / 2 - 1] + im[c / 2]);
            }
        }
        fin[2 * e] = vr;
        fin[2 * e + 1] = vi;
        mysurv += sqrt(vr * vr + vi * vi) > half_theta;
    }
    __syncthreads();
    if (tid == 0) S.flag = 0;
    __syncthreads();
    if (mysurv) atomicAdd(&S.flag, mysurv);
    __syncthreads();
    const uint32_t nsurv = S.flag;
    uint64_t* oidx = D.out_idx + (uint64_t)sig * D.cap;
    double* oval = D.out_val + (uint64_t)sig * D.cap * 2;
    uint32_t flags = st[ST_FLAGS];
    uint32_t nout;
    if (nsurv <= D.cap) {
        // ordered compaction: thread t takes a contiguous chunk of entries
        const uint32_t chunk = (zc + kThreads - 1) / kThreads;
        const uint32_t e0 = tid * chunk;
        const uint32_t e1 = e0 + chunk < zc ? e0 + chunk : zc;
        uint32_t cnt = 0;
        for (uint32_t e = e0; e < e1; ++e)
            cnt += sqrt(fin[2 * e] * fin[2 * e] + fin[2 * e + 1] * fin[2 * e + 1]) > half_theta;
        uint32_t pre;
        block_exclusive_scan(cnt, S.scan, &pre);
        for (uint32_t e = e0; e < e1; ++e) {
            const double vr = fin[2 * e], vi = fin[2 * e + 1];
            if (sqrt(vr * vr + vi * vi) > half_theta) {
                oidx[pre] = zi[e];
                oval[2 * pre] = vr * D.out_scale;
                oval[2 * pre + 1] = vi * D.out_scale;
                ++pre;
            }
        }
        nout = nsurv;
    } else {
        // top-cap by (|v| desc, index asc): |v| > 0, so its IEEE bits order like |v|
        flags |= 1u;
        const uint32_t N = pow2_at_least(zc);
        // key = ~(bits(|v|) >> 12) << 13 | e: 51 magnitude bits, ties by entry
        for (uint32_t e = tid; e < N; e += kThreads) {
            if (e < zc) {
                const double vr = fin[2 * e], vi = fin[2 * e + 1];
                const double m = sqrt(vr * vr + vi * vi);
                const uint64_t mb = (uint64_t)__double_as_longlong(m) >> 12;
                S.key[e] = ((~mb & ((1ull << 51) - 1)) << 13) | e;
            } else {
                S.key[e] = kNone;
            }
        }
        bitonic_sort_u64(S.key, N);
        // keep the first cap entries, re-sort them by entry (= index order)
        for (uint32_t q = tid; q < N; q += kThreads) {
            if (q >= D.cap) S.key[q] = kNone;
            else S.key[q] = S.key[q] & 0x1FFFull;
        }
        bitonic_sort_u64(S.key, N);
        for (uint32_t q = tid; q < D.cap; q += kThreads) {
            const uint32_t e = (uint32_t)S.key[q];
            oidx[q] = zi[e];
            oval[2 * q] = fin[2 * e] * D.out_scale;
            oval[2 * q + 1] = fin[2 * e + 1] * D.out_scale;
        }
        nout = D.cap;
    }
    __syncthreads();
    for (uint32_t q = nout + tid; q < D.cap; q += kThreads) {
        oidx[q] = 0;
        oval[2 * q] = 0.0;
        oval[2 * q + 1] = 0.0;
    }
    if (tid == 0) {
        D.out_count[sig] = nout;
        st[ST_FLAGS] = flags;
        if (D.out_info) {
            D.out_info[(uint64_t)sig * 4 + SFFT_INFO_ROUNDS] = R;
            D.out_info[(uint64_t)sig * 4 + SFFT_INFO_FLAGS] = flags;
            D.out_info[(uint64_t)sig * 4 + SFFT_INFO_ZHAT] = zc;
            D.out_info[(uint64_t)sig * 4 + SFFT_INFO_LOCATED] = 0;
        }
    }
}

// ------------------------------------------------------------------ general
// General (noisy) recovery, Algorithms 2 and 3.  One workgroup per signal
// runs the SparseFFT rounds on raw bins computed up front: LocateSignal with
// one thread per bin carrying that bin's region through every LocateInner
// level, EstimateValues medians over the candidates, the top-3k_r selection
// and the merge into zhat; the finish kernel re-estimates every zhat entry
// over all EstimateValues measurements in FP64.

constexpr uint32_t kMaxMeas = 64;   // measurements per entry in the final re-estimation

struct GenShared {
    DecodeShared d;
    uint16_t binfirst[kMaxZ];       // first sorted position of each bin, 0xFFFF = none
};

__device__ __forceinline__ const double* gen_raw(const GeneralArgs& G, uint32_t sig, uint32_t slot, uint32_t a) {
    return G.raw + (((uint64_t)sig * G.nslots + slot) * 2 + a) * (uint64_t)G.Bmax * 2;
}

// Sort the zhat entries by bin of (sigma, b, B) and index each bin's first entry.
__device__ void index_bins(GenShared& S, const uint64_t* zi, uint32_t zc, uint64_t sigma, uint64_t b, uint64_t n,
                           uint32_t B) {
    sort_entries_by_bin(S.d, zi, zc, sigma, b, n, B);
    for (uint32_t j = threadIdx.x; j < B; j += kThreads) S.binfirst[j] = 0xFFFF;
    __syncthreads();
    for (uint32_t p = threadIdx.x; p < zc; p += kThreads) {
        const uint32_t h = (uint32_t)(S.d.key[p] >> kKeyBinShift);
        if (p == 0 || (uint32_t)(S.d.key[p - 1] >> kKeyBinShift) != h) S.binfirst[h] = (uint16_t)p;
    }
    __syncthreads();
}

// HashToBins step 4 for one bin: u_h - sum over the zhat entries of bin h,
// in ascending index order, of G'_{-o(i)} zhat_i omega^{shift sigma i}.
__device__ cx<double> corrected_bin(const GenShared& S, const double* rawv, uint32_t h, uint64_t shift,
                                    const uint64_t* zi, const double* zv, uint32_t zc, uint64_t sigma, uint64_t b,
                                    uint64_t n, uint32_t B, const WindowShape& ws) {
    cx<double> u{rawv[2 * h], rawv[2 * h + 1]};
    const uint32_t p0 = S.binfirst[h];
    if (p0 == 0xFFFF) return u;
    const uint64_t mask = n - 1;
    const uint64_t as = (shift * sigma) & mask;
    for (uint32_t q = p0; q < zc && (uint32_t)(S.d.key[q] >> kKeyBinShift) == h; ++q) {
        const uint32_t e = (uint32_t)(S.d.key[q] & kEntryMask);
        const uint64_t i = zi[e];
        const BinOffset bo = bin_offset(i, sigma, b, n, B);
        const double gp = gprime(-bo.o, n, B, ws);
        const cx<double> c0{gp * zv[2 * e], gp * zv[2 * e + 1]};
        u = csub(u, cmul(c0, omega_d((as * i) & mask, n)));
    }
    return u;
}

__device__ __forceinline__ double phase_of(cx<double> u, cx<double> u2) {
    const double zr = u.r * u2.r + u.i * u2.i;
    const double zi = u.i * u2.r - u.r * u2.i;
    double ph = atan2(zi, zr);
    if (ph < 0.0) ph += 6.283185307179586;
    return ph;
}

// Median of c values (re and im separately; even counts average the middle two).
__device__ cx<double> median_cx(double* re, double* im, uint32_t c) {
    for (uint32_t q = 1; q < c; ++q) {
        const double a = re[q], bq = im[q];
        int32_t s = (int32_t)q - 1;
        while (s >= 0 && re[s] > a) { re[s + 1] = re[s]; --s; }
        re[s + 1] = a;
        s = (int32_t)q - 1;
        while (s >= 0 && im[s] > bq) { im[s + 1] = im[s]; --s; }
        im[s + 1] = bq;
    }
    if (c & 1) return {re[c / 2], im[c / 2]};
    return {0.5 * (re[c / 2 - 1] + re[c / 2]), 0.5 * (im[c / 2 - 1] + im[c / 2])};
}

// Magnitude-descending sort key with 13 bits of tie-break slot (ascending).
__device__ __forceinline__ uint64_t mag_key(double vr, double vi, uint32_t slot) {
    const double m = sqrt(vr * vr + vi * vi);
    const uint64_t mb = (uint64_t)__double_as_longlong(m) >> 12;
    return ((~mb & ((1ull << 51) - 1)) << 13) | slot;
}

// One SparseFFT round: LocateSignal, EstimateValues, zhat update.
__device__ void general_round(const GeneralArgs& G, GenShared& S, uint32_t sig, uint32_t r, uint64_t seed) {
    const uint32_t tid = threadIdx.x;
    const RoundDev g = G.geom[r];
    const GenRoundDev& gr = G.groundv[r];
    const uint64_t n = G.n, mask = n - 1;
    const uint32_t B = g.B;
    uint32_t* st = G.state + (uint64_t)sig * kStateWords;
    const uint32_t zc = st[ST_ZCOUNT];
    const uint32_t zb = st[ST_ZBUF];
    const uint64_t* zi = G.zidx + ((uint64_t)sig * 2 + zb) * G.capz;
    const double* zv = G.zval + ((uint64_t)sig * 2 + zb) * G.capz * 2;
    uint64_t* cand = G.cand_i + (uint64_t)sig * G.Bmax;
    double* candv = G.cand_v + (uint64_t)sig * G.Bmax * 2;
    uint32_t* candn = G.cand_n + (uint64_t)sig * G.Bmax;
    const double two_pi = 6.283185307179586;

    // ---- LocateSignal (Algorithm 3): one (sigma, b); regions per bin
    {
        const uint64_t scale = 1ull << kFracBits;
        const uint64_t modfp = n << kFracBits;
        const uint64_t mmask = modfp - 1;
        const uint64_t sigma = draw_sigma(seed, n, r, 0, 0);
        const uint64_t b = draw_b(seed, n, r, 0, 0);
        const uint64_t sinv = inverse_odd(sigma) & mask;
        const uint64_t sbs = ((sigma * b) & mask) << kFracBits;
        const double tol = G.s * 3.141592653589793;
        index_bins(S, zi, zc, sigma, b, n, B);
        for (uint32_t j = tid; j < B; j += kThreads) {
            uint64_t l = ((uint64_t)j * (n / B) * scale + modfp - (n / (2 * (uint64_t)B)) * scale) & mmask;
            bool alive = true;
            for (uint32_t D = 1; D <= gr.nlev && alive; ++D) {
                const uint64_t W = gr.Wfp[D - 1];
                const uint64_t half = W / (2 * G.t);
                const uint64_t step = W / G.t;
                uint8_t votes[kMaxT];
                for (uint32_t qq = 0; qq < G.t; ++qq) votes[qq] = 0;
                for (uint32_t q = 0; q < G.R_loc; ++q) {
                    const uint64_t a = draw_a(seed, n, r, D, q);
                    const uint64_t beta = draw_beta(seed, gr.blo[D - 1], gr.bhi[D - 1], r, D, q);
                    const uint32_t slot = gr.slot0 + (D - 1) * G.R_loc + q;
                    const cx<double> u = corrected_bin(S, gen_raw(G, sig, slot, 0), j, a, zi, zv, zc, sigma, b, n, B, g.ws);
                    const cx<double> u2 = corrected_bin(S, gen_raw(G, sig, slot, 1), j, (a + beta) & mask, zi, zv, zc,
                                                        sigma, b, n, B, g.ws);
                    const double c = phase_of(u, u2);
                    for (uint32_t qq = 0; qq < G.t; ++qq) {
                        const uint64_t M = (l + (2 * (uint64_t)qq + 1) * half) & mmask;
                        const uint64_t num = (beta * ((M + sbs) & mmask)) & mmask;
                        const double ang = two_pi * (double)num / (double)modfp;
                        const double d = fabs(ang - c);
                        const double dist = d < two_pi - d ? d : two_pi - d;
                        votes[qq] += dist < tol;
                    }
                }
                uint32_t first = G.t;
                for (uint32_t qq = 0; qq < G.t; ++qq)
                    if (2u * votes[qq] > G.R_loc) {
                        first = qq;
                        break;
                    }
                if (first == G.t) alive = false;
                else l = (l + first * step) & mmask;
            }
            uint64_t ci = kNone;
            if (alive) {
                const uint64_t pos = ((l + scale - 1) >> kFracBits) & mask;
                ci = (sinv * pos + b) & mask;
            }
            cand[j] = ci;
        }
    }
    __syncthreads();
    // L: sorted, unique candidate indices
    const uint32_t NB = pow2_at_least(B);
    for (uint32_t j = tid; j < NB; j += kThreads) S.d.key[j] = j < B ? cand[j] : kNone;
    bitonic_sort_u64(S.d.key, NB);
    {
        const uint32_t chunk = (NB + kThreads - 1) / kThreads;
        const uint32_t p0 = tid * chunk, p1 = p0 + chunk < NB ? p0 + chunk : NB;
        uint32_t cnt = 0;
        for (uint32_t p = p0; p < p1; ++p)
            cnt += S.d.key[p] != kNone && (p == 0 || S.d.key[p] != S.d.key[p - 1]);
        uint32_t pre;
        const uint32_t total = block_exclusive_scan(cnt, S.d.scan, &pre);
        for (uint32_t p = p0; p < p1; ++p)
            if (S.d.key[p] != kNone && (p == 0 || S.d.key[p] != S.d.key[p - 1])) cand[pre++] = S.d.key[p];
        if (tid == 0) S.d.flag = total;
        __syncthreads();
    }
    const uint32_t nL = S.d.flag;
    __syncthreads();

    // ---- EstimateValues (Algorithm 2): R_est fresh hashings, medians
    for (uint32_t c = tid; c < nL; c += kThreads) candn[c] = 0;
    for (uint32_t e = 0; e < G.R_est; ++e) {
        const uint64_t sigma = draw_sigma(seed, n, r, LEVEL_EST, e);
        const uint64_t a = draw_a(seed, n, r, LEVEL_EST, e);
        const uint64_t b = draw_b(seed, n, r, LEVEL_EST, e);
        const uint32_t slot = gr.slot0 + gr.nloc + e;
        __syncthreads();
        index_bins(S, zi, zc, sigma, b, n, B);
        const double* rawv = gen_raw(G, sig, slot, 0);
        for (uint32_t c = tid; c < nL; c += kThreads) {
            const uint64_t i = cand[c];
            const BinOffset bo = bin_offset(i, sigma, b, n, B);
            const double gp = gprime(-bo.o, n, B, g.ws);
            if (gp < G.g_min) continue;
            const cx<double> u = corrected_bin(S, rawv, bo.h, a, zi, zv, zc, sigma, b, n, B, g.ws);
            const uint64_t p = (((a * sigma) & mask) * i) & mask;
            const cx<double> v = cmul(u, omega_d((n - p) & mask, n));
            const uint32_t k = candn[c];
            double* dst = G.cand_e + (((uint64_t)sig * G.R_est + k) * G.Bmax + c) * 2;
            dst[0] = v.r / gp;
            dst[1] = v.i / gp;
            candn[c] = k + 1;
        }
    }
    __syncthreads();
    for (uint32_t c = tid; c < nL; c += kThreads) {
        const uint32_t k = candn[c];
        if (k == 0) continue;
        double re[kMaxMeas], im[kMaxMeas];
        for (uint32_t q = 0; q < k; ++q) {
            const double* src = G.cand_e + (((uint64_t)sig * G.R_est + q) * G.Bmax + c) * 2;
            re[q] = src[0];
            im[q] = src[1];
        }
        const cx<double> m = median_cx(re, im, k);
        candv[2 * c] = m.r;
        candv[2 * c + 1] = m.i;
    }
    __syncthreads();
    // top-k' by (|w| desc, index asc); candidates are in index order
    const uint32_t kprime = 3 * gr.k_r;
    const uint32_t NL = pow2_at_least(nL > 0 ? nL : 1);
    for (uint32_t c = tid; c < NL; c += kThreads)
        S.d.key[c] = (c < nL && candn[c] > 0) ? mag_key(candv[2 * c], candv[2 * c + 1], c) : kNone;
    bitonic_sort_u64(S.d.key, NL);
    for (uint32_t q = tid; q < NL; q += kThreads) {
        const uint64_t k = S.d.key[q];
        if (q >= kprime || k == kNone) {
            S.d.key[q] = kNone;
        } else {
            const uint32_t c = (uint32_t)(k & 0x1FFFull);
            S.d.key[q] = (cand[c] << kCandShift) | c;
        }
    }
    bitonic_sort_u64(S.d.key, NL);
    merge_candidates(S.d, NL, candv, G.zidx, G.zval, sig, G.capz, st);
    if (tid == 0) {
        st[ST_ROUNDS] = r + 1;
        st[ST_LASTJ] = nL;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kThreads) k_general_decode(GeneralArgs G, uint32_t r_begin, uint32_t r_end) {
    __shared__ GenShared S;
    const uint32_t sig = blockIdx.x;
    const uint64_t seed = G.seeds ? G.seeds[sig] : G.plan_seed;
    for (uint32_t r = r_begin; r < r_end; ++r) {
        __syncthreads();
        general_round(G, S, sig, r, seed);
    }
}

// Final FP64 re-estimation over every EstimateValues measurement of every
// round (isolated measurements first), then the top-cap entries by magnitude
// in ascending index order.
__global__ void __launch_bounds__(kThreads) k_general_finish(GeneralArgs G) {
    __shared__ GenShared S;
    const uint32_t tid = threadIdx.x;
    const uint32_t sig = blockIdx.x;
    const uint64_t seed = G.seeds ? G.seeds[sig] : G.plan_seed;
    uint32_t* st = G.state + (uint64_t)sig * kStateWords;
    const uint64_t n = G.n, mask = n - 1;
    const uint32_t zc = st[ST_ZCOUNT];
    const uint32_t zb = st[ST_ZBUF];
    const uint32_t R = st[ST_ROUNDS];
    const uint64_t* zi = G.zidx + ((uint64_t)sig * 2 + zb) * G.capz;
    const double* zv = G.zval + ((uint64_t)sig * 2 + zb) * G.capz * 2;
    const uint32_t nmeas = G.R * G.R_est;
    double* est = G.est + (uint64_t)sig * G.capz * nmeas * 2;
    uint32_t* ecount = G.ecount + (uint64_t)sig * G.capz;
    double* gtmp = G.gtmp + (uint64_t)sig * G.capz;
    double* fin = G.fin + (uint64_t)sig * G.capz * 2;
    for (uint32_t e = tid; e < zc; e += kThreads) ecount[e] = 0;
    for (uint32_t r = 0; r < R; ++r) {
        const RoundDev g = G.geom[r];
        const GenRoundDev& gr = G.groundv[r];
        const uint32_t B = g.B;
        for (uint32_t m = 0; m < G.R_est; ++m) {
            const uint64_t sigma = draw_sigma(seed, n, r, LEVEL_EST, m);
            const uint64_t a = draw_a(seed, n, r, LEVEL_EST, m);
            const uint64_t b = draw_b(seed, n, r, LEVEL_EST, m);
            const double* rawv = gen_raw(G, sig, gr.slot0 + gr.nloc + m, 0);
            const uint64_t as = (a * sigma) & mask;
            __syncthreads();
            for (uint32_t e = tid; e < zc; e += kThreads) {
                const BinOffset bo = bin_offset(zi[e], sigma, b, n, B);
                gtmp[e] = gprime(-bo.o, n, B, g.ws);
            }
            index_bins(S, zi, zc, sigma, b, n, B);
            for (uint32_t p = tid; p < zc; p += kThreads) {
                const uint32_t e = (uint32_t)(S.d.key[p] & kEntryMask);
                const double ge = gtmp[e];
                if (ge < G.g_min) continue;
                const uint32_t h = (uint32_t)(S.d.key[p] >> kKeyBinShift);
                const uint32_t s0 = S.binfirst[h];
                cx<double> others{0.0, 0.0};
                uint32_t members = 0;
                for (uint32_t q = s0; q < zc && (uint32_t)(S.d.key[q] >> kKeyBinShift) == h; ++q) {
                    ++members;
                    const uint32_t e2 = (uint32_t)(S.d.key[q] & kEntryMask);
                    if (e2 == e) continue;
                    const cx<double> c0{gtmp[e2] * zv[2 * e2], gtmp[e2] * zv[2 * e2 + 1]};
                    others = cadd(others, cmul(c0, omega_d((as * zi[e2]) & mask, n)));
                }
                const cx<double> u = csub(cx<double>{rawv[2 * h], rawv[2 * h + 1]}, others);
                const uint64_t pe = (as * zi[e]) & mask;
                const cx<double> v = cmul(u, omega_d((n - pe) & mask, n));
                const uint32_t c = ecount[e];
                const uint32_t na = c & 0xFFFFu, nb = c >> 16;
                const uint32_t slot = members == 1 ? na : nmeas - 1 - nb;
                est[((uint64_t)e * nmeas + slot) * 2] = v.r / ge;
                est[((uint64_t)e * nmeas + slot) * 2 + 1] = v.i / ge;
                ecount[e] = members == 1 ? c + 1 : c + (1u << 16);
            }
        }
    }
    __syncthreads();
    for (uint32_t e = tid; e < zc; e += kThreads) {
        const uint32_t na = ecount[e] & 0xFFFFu, nb = ecount[e] >> 16;
        const uint32_t c = na ? na : nb;
        const uint32_t first = na ? 0u : nmeas - nb;
        cx<double> v{zv[2 * e], zv[2 * e + 1]};
        if (c > 0) {
            double re[kMaxMeas], im[kMaxMeas];
            for (uint32_t q = 0; q < c; ++q) {
                re[q] = est[((uint64_t)e * nmeas + first + q) * 2];
                im[q] = est[((uint64_t)e * nmeas + first + q) * 2 + 1];
            }
            v = median_cx(re, im, c);
        }
        fin[2 * e] = v.r;
        fin[2 * e + 1] = v.i;
    }
    __syncthreads();
    // top cap by (|v| desc, index asc), output in index order
    const uint32_t N = pow2_at_least(zc > 0 ? zc : 1);
    for (uint32_t e = tid; e < N; e += kThreads) S.d.key[e] = e < zc ? mag_key(fin[2 * e], fin[2 * e + 1], e) : kNone;
    bitonic_sort_u64(S.d.key, N);
    const uint32_t nout = zc < G.cap ? zc : G.cap;
    for (uint32_t q = tid; q < N; q += kThreads) S.d.key[q] = q < nout ? (S.d.key[q] & 0x1FFFull) : kNone;
    bitonic_sort_u64(S.d.key, N);
    uint64_t* oidx = G.out_idx + (uint64_t)sig * G.cap;
    double* oval = G.out_val + (uint64_t)sig * G.cap * 2;
    for (uint32_t q = tid; q < G.cap; q += kThreads) {
        if (q < nout) {
            const uint32_t e = (uint32_t)S.d.key[q];
            oidx[q] = zi[e];
            oval[2 * q] = fin[2 * e] * G.out_scale;
            oval[2 * q + 1] = fin[2 * e + 1] * G.out_scale;
        } else {
            oidx[q] = 0;
            oval[2 * q] = 0.0;
            oval[2 * q + 1] = 0.0;
        }
    }
    if (tid == 0) {
        G.out_count[sig] = nout;
        if (G.out_info) {
            G.out_info[(uint64_t)sig * 4 + SFFT_INFO_ROUNDS] = R;
            G.out_info[(uint64_t)sig * 4 + SFFT_INFO_FLAGS] = st[ST_FLAGS];
            G.out_info[(uint64_t)sig * 4 + SFFT_INFO_ZHAT] = zc;
            G.out_info[(uint64_t)sig * 4 + SFFT_INFO_LOCATED] = st[ST_LASTJ];
        }
    }
}

// ------------------------------------------------------------------ launch --
size_t h2b_pair_lds_bytes(uint32_t Bmax, uint64_t max_mcount, bool acc_f64) {
    const size_t csz = acc_f64 ? 16 : 8;
    const size_t slots = Bmax >= kThreads ? Bmax : kThreads;
    return (2 * slots + max_mcount) * csz;
}

// Dynamic LDS above 64 KiB needs the per-kernel opt-in (gfx950 has 160 KiB).
template <class K>
static hipError_t allow_lds(K kernel, size_t lds) {
    if (lds <= 64 * 1024) return hipSuccess;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

template <class TIn, class TA>
static hipError_t launch_pair_t(const H2BArgs& a, size_t lds, uint32_t grid, hipStream_t s) {
    hipError_t e = allow_lds(k_h2b_pair<TIn, TA>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_h2b_pair<TIn, TA>), dim3(grid), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

template <class TIn, class TA>
static hipError_t launch_split_t(const H2BArgs& a, uint32_t round, size_t lds, hipStream_t s) {
    hipError_t e = allow_lds(k_h2b_split<TIn, TA>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_h2b_split<TIn, TA>), dim3(a.parts), dim3(kThreads), lds, s, a, round);
    return hipGetLastError();
}

hipError_t launch_h2b_pair(const H2BArgs& a, bool in_c128, bool acc_f64, hipStream_t s) {
    // LDS: two fold arrays of max(Bmax, threads) plus the modulation table
    const size_t lds = h2b_pair_lds_bytes(a.Bmax, a.mcap, acc_f64);
    const uint32_t grid = a.explicit_job ? 1u : (a.jobs ? a.count * a.njobs : a.count * a.nrounds);
    if (in_c128) return acc_f64 ? launch_pair_t<double2, double>(a, lds, grid, s)
                                : launch_pair_t<double2, float>(a, lds, grid, s);
    return acc_f64 ? launch_pair_t<float2, double>(a, lds, grid, s) : launch_pair_t<float2, float>(a, lds, grid, s);
}

hipError_t launch_h2b_split(const H2BArgs& a, uint32_t round, bool in_c128, bool acc_f64, hipStream_t s) {
    const size_t lds = h2b_pair_lds_bytes(a.Bmax, a.mcap, acc_f64);
    if (in_c128) return acc_f64 ? launch_split_t<double2, double>(a, round, lds, s)
                                : launch_split_t<double2, float>(a, round, lds, s);
    return acc_f64 ? launch_split_t<float2, double>(a, round, lds, s) : launch_split_t<float2, float>(a, round, lds, s);
}

hipError_t launch_h2b_reduce(const H2BArgs& a, uint32_t round, bool acc_f64, hipStream_t s) {
    const size_t lds = 2 * (size_t)a.Bmax * (acc_f64 ? 16 : 8);
    hipError_t e = acc_f64 ? allow_lds(k_h2b_reduce<double>, lds) : allow_lds(k_h2b_reduce<float>, lds);
    if (e != hipSuccess) return e;
    if (acc_f64) hipLaunchKernelGGL((k_h2b_reduce<double>), dim3(1), dim3(kThreads), lds, s, a, round);
    else hipLaunchKernelGGL((k_h2b_reduce<float>), dim3(1), dim3(kThreads), lds, s, a, round);
    return hipGetLastError();
}

hipError_t launch_exact_init(const DecodeArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_exact_init, dim3((a.count + kThreads - 1) / kThreads), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_exact_decode(const DecodeArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_exact_decode, dim3(a.count), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_exact_finish(const DecodeArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_exact_finish, dim3(a.count), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_general_decode(const GeneralArgs& a, uint32_t r_begin, uint32_t r_end, hipStream_t s) {
    hipLaunchKernelGGL(k_general_decode, dim3(a.count), dim3(kThreads), 0, s, a, r_begin, r_end);
    return hipGetLastError();
}

hipError_t launch_general_finish(const GeneralArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_general_finish, dim3(a.count), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace sfft
