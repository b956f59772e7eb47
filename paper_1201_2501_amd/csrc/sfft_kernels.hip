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
//  * k_h2b_pstream   stream mode of the batched exact pair: each of `parts`
//                    workgroups per (signal, round) reads a contiguous share
//                    of the whole signal and keeps the samples that fall in
//                    the window (for windows that cover a large fraction of
//                    a small signal); its partial folds go to k_h2b_rsplit
//  * k_h2b_psplit,   the batched exact pair split over `parts` workgroups per
//    k_h2b_rsplit    (signal, round) by window range, then one workgroup per
//                    (signal, round) sums the partials in part order,
//                    modulates, transforms and stores the raw bins: for small
//                    batches, where one workgroup per hashing leaves the chip
//                    idle and a long window is walked by one CU
// The decoders (exact and general mode) are in sfft_decode.hip.
#include "sfft_pair.hpp"

namespace sfft {


// (signal, round offset) of job j of a batched exact pair launch, in the
// plan's workgroup order: round-major; signal-major; or signal-major within
// each XCD (job j runs on XCD j mod 8, which takes the signals s = j mod 8).
__device__ __forceinline__ void pair_job(const H2BArgs& A, uint32_t j, uint32_t* sig, uint32_t* rr) {
    const uint32_t C = A.count, R = A.nrounds;
    if (A.order == 2 && (C & 7u) == 0) {
        const uint32_t q = j >> 3, s8 = q / R;
        *rr = q - s8 * R;
        *sig = s8 * 8 + (j & 7u);
    } else if (A.order != 0) {
        *sig = j / R;
        *rr = j - *sig * R;
    } else {
        *rr = j / C;
        *sig = j - *rr * C;
    }
}

// TRI: the exact batched pair plus a third hashing at shift A.gamma (the
// multi-shift phase refinement), stored in the round's third raw-bin slot.
template <class TIn, class TA, uint32_t NT, bool TRI>
__global__ void __launch_bounds__(NT) k_h2b_pair(H2BArgs A) {
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
        uint32_t rr;
        pair_job(A, blockIdx.x, &sig, &rr);
        // the method stops a signal after `patience` empty rounds: its later
        // hashings are never decoded
        if (A.state && A.state[(uint64_t)sig * kStateWords + ST_DONE]) return;
        r = A.round_lo + rr;
        ro = r;
        const uint64_t seed = A.seeds ? A.seeds[sig] : A.plan_seed;
        sigma = draw_sigma(seed, n, r);
        b = draw_b(seed, n, r);
        a = 0;
        beta = 1;
    }
    const RoundDev g = A.geom[r];
    const TIn* x = A.xptrs ? reinterpret_cast<const TIn*>(A.xptrs[sig])
                           : reinterpret_cast<const TIn*>(A.x) + (uint64_t)sig * A.sig_stride;
    const TA* G = reinterpret_cast<const TA*>(A.gtab) + g.gofs;
    const auto* tw = reinterpret_cast<const typename TwTraits<TA>::V*>(A.tw);
    const uint32_t B = g.B;
    const uint32_t parts = B >= NT ? 1u : NT / B;
    cx<TA>* VA = reinterpret_cast<cx<TA>*>(smem);
    cx<TA>* VB = VA + parts * B;
    cx<TA>* VC = VB + parts * B;                  // TRI: the third hashing and a zero companion
    cx<TA>* VD = VC + parts * B;
    cx<TA>* M = TRI ? VD + parts * B : VC;
    for (uint32_t q = threadIdx.x; q < parts * B; q += NT) {
        VA[q] = cx<TA>{0, 0};
        VB[q] = cx<TA>{0, 0};
        if (TRI) {
            VC[q] = cx<TA>{0, 0};
            VD[q] = cx<TA>{0, 0};
        }
    }
    accumulate_pair<TIn, TA, NT, TRI>(x, G, VA, VB, M, n, sigma, a, beta, b, B, g.logB, g.w, g.t0,
                                      INT64_MIN / 4, INT64_MAX / 4, parts, VC, A.gamma);
    __syncthreads();
    finalize_folds<TA, NT>(VA, VB, n, sigma, b, beta, B, parts);
    if (TRI) finalize_folds<TA, NT>(VD, VC, n, sigma, b, A.gamma, B, parts);
    __syncthreads();
    lds_fft2<TA, NT>(VA, VB, B, A.Bmax, tw);
    if (TRI) lds_fft2<TA, NT>(VD, VC, B, A.Bmax, tw);
    double* out0 = A.raw + (((uint64_t)sig * A.raw_rounds + ro) * A.nhash) * (uint64_t)A.Bmax * 2;
    store_bins<TA, NT>(VA, VB, B, g.logB, A.Bmax, beta, tw, A.sqrt_n, out0, out0 + 2 * (uint64_t)A.Bmax);
    if (TRI)
        store_bins<TA, NT>(VD, VC, B, g.logB, A.Bmax, A.gamma, tw, A.sqrt_n, nullptr,
                           out0 + 4 * (uint64_t)A.Bmax);
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
    accumulate_pair<TIn, TA, kThreads>(x, G, VA, VB, M, n, sigma, a, beta, b, B, g.logB, g.w, g.t0, Llo, Lhi,
                                       parts);
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
    finalize_folds<TA, kThreads>(VA, VB, A.n, A.sigma, A.b, A.beta, B, 1);
    __syncthreads();
    lds_fft2<TA, kThreads>(VA, VB, B, A.Bmax, tw);
    double* out0 = A.raw + ((uint64_t)round * A.nhash) * (uint64_t)A.Bmax * 2;
    store_bins<TA, kThreads>(VA, VB, B, g.logB, A.Bmax, A.beta, tw, A.sqrt_n, out0, out0 + 2 * (uint64_t)A.Bmax);
}

// Exact batched mode with a split hashing: the (signal, round) of job j of a
// pair launch (j = round offset * count + signal) and whether its signal has
// stopped decoding.
struct SplitJob {
    uint32_t sig, r;
    uint64_t sigma, b;
};

__device__ __forceinline__ bool split_job(const H2BArgs& A, uint32_t job, SplitJob& J) {
    uint32_t rr;
    pair_job(A, job, &J.sig, &rr);
    if (A.state && A.state[(uint64_t)J.sig * kStateWords + ST_DONE]) return false;
    J.r = A.round_lo + rr;
    const uint64_t seed = A.seeds ? A.seeds[J.sig] : A.plan_seed;
    J.sigma = draw_sigma(seed, A.n, J.r);
    J.b = draw_b(seed, A.n, J.r);
    return true;
}

// Stage 1: part blockIdx.x of job blockIdx.y accumulates its share of the
// window's segments (shifts 0 and 1) and writes unmodulated partial folds
// [job][part][2][B] (complex128, slots of Bmax).
template <class TIn, class TA>
__global__ void __launch_bounds__(kThreads) k_h2b_psplit(H2BArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t job = blockIdx.y, part = blockIdx.x;
    SplitJob J;
    if (!split_job(A, job, J)) return;
    const uint64_t n = A.n;
    const RoundDev g = A.geom[J.r];
    const TIn* x = A.xptrs ? reinterpret_cast<const TIn*>(A.xptrs[J.sig])
                           : reinterpret_cast<const TIn*>(A.x) + (uint64_t)J.sig * A.sig_stride;
    const TA* G = reinterpret_cast<const TA*>(A.gtab) + g.gofs;
    const uint32_t B = g.B;
    const uint32_t sub = B >= kThreads ? 1u : kThreads / B;
    cx<TA>* VA = reinterpret_cast<cx<TA>*>(smem);
    cx<TA>* VB = VA + sub * B;
    cx<TA>* M = VB + sub * B;
    for (uint32_t q = threadIdx.x; q < sub * B; q += kThreads) {
        VA[q] = cx<TA>{0, 0};
        VB[q] = cx<TA>{0, 0};
    }
    // segments L of the window at shifts 0 and 1, cut into A.parts ranges; the
    // first and last ranges are open so that the ranges cover every L
    const int64_t iB = (int64_t)B;
    const int64_t Lmin = floordiv(g.t0 - 1 - (iB - 1), iB);
    const int64_t Lmax = floordiv(g.t0 + (int64_t)g.w - 1, iB);
    const int64_t chunk = (Lmax - Lmin + (int64_t)A.parts) / (int64_t)A.parts;
    const int64_t lo = part == 0 ? INT64_MIN / 4 : Lmin + (int64_t)part * chunk;
    const int64_t hi = part + 1 == A.parts ? INT64_MAX / 4 : Lmin + (int64_t)(part + 1) * chunk - 1;
    accumulate_pair<TIn, TA, kThreads>(x, G, VA, VB, M, n, J.sigma, 0, 1, J.b, B, g.logB, g.w, g.t0, lo, hi, sub);
    __syncthreads();
    double* out = A.partial + ((uint64_t)job * A.parts + part) * 4 * (uint64_t)A.Bmax;
    for (uint32_t r = threadIdx.x; r < B; r += kThreads) {
        cx<TA> sa = VA[r], sb = VB[r];
        for (uint32_t p = 1; p < sub; ++p) {
            sa = cadd(sa, VA[p * B + r]);
            sb = cadd(sb, VB[p * B + r]);
        }
        out[2 * r] = (double)sa.r;
        out[2 * r + 1] = (double)sa.i;
        out[2 * B + 2 * r] = (double)sb.r;
        out[2 * B + 2 * r + 1] = (double)sb.i;
    }
}

// Stage 1 of a stream-mode pair (k_h2b_pstream, then k_h2b_rsplit): part
// blockIdx.x of job blockIdx.y reads its share of the signal contiguously
// instead of gathering the window.  Sample m sits at t_A = sigma^{-1} m
// (mod n, taken in [-n/2, n/2)) of the shift-0 hashing; every m of one
// residue class rho = m mod B has the same residue r = t_A mod B (sigma is
// odd), so the thread that owns class rho owns residue r and adds, in
// ascending m, the samples whose t_A lies in the pair's window rows:
// G_{t_A - t0} M_L x_m to hashing A and G_{t_A + 1 - t0} M_L x_m to hashing
// B, as accumulate_pair does (the same partial folds, added in another
// order).  With B < 256 the block's threads split each class into
// 256 / B lanes of interleaved m, summed in lane order at the end; each
// iteration of a block then reads 256 consecutive samples.
template <class TIn, class TA>
__global__ void __launch_bounds__(kThreads) k_h2b_pstream(H2BArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t job = blockIdx.y, part = blockIdx.x;
    SplitJob J;
    if (!split_job(A, job, J)) return;
    const uint64_t n = A.n, mask = n - 1, half = n >> 1;
    const RoundDev g = A.geom[J.r];
    const TIn* x = A.xptrs ? reinterpret_cast<const TIn*>(A.xptrs[J.sig])
                           : reinterpret_cast<const TIn*>(A.x) + (uint64_t)J.sig * A.sig_stride;
    const TA* G = reinterpret_cast<const TA*>(A.gtab) + g.gofs;
    const uint32_t B = g.B;
    const uint32_t lanes = B >= kThreads ? 1u : kThreads / B;
    cx<TA>* VA = reinterpret_cast<cx<TA>*>(smem);
    cx<TA>* VB = VA + lanes * B;
    cx<TA>* M = VB + lanes * B;
    const int64_t iB = (int64_t)B, iw = (int64_t)g.w;
    // window rows of t_A in [t0 - 1, t0 + w): the pair at shifts 0 and 1
    const int64_t Llo = floordiv(g.t0 - 1, iB);
    const int64_t Lhi = floordiv(g.t0 + iw - 1, iB);
    const uint64_t c = (J.sigma * J.b) & mask;
    const uint64_t cB = (c * (uint64_t)B) & mask;
    for (int64_t L = Llo + threadIdx.x; L <= Lhi; L += kThreads)
        M[L - Llo] = to_cx<TA>(omega_d((cB * (uint64_t)L) & mask, n));
    __syncthreads();
    const uint64_t sinv = inverse_odd(J.sigma) & mask;
    const uint64_t rows = n / B;                                  // samples per class
    const uint64_t per = rows / A.parts;                          // parts divide rows (powers of two)
    const uint64_t j0 = (uint64_t)part * per;
    const uint32_t nslot = lanes * B;
    for (uint32_t slot = threadIdx.x; slot < nslot; slot += kThreads) {
        const uint32_t rho = slot % B, lane = slot / B;
        const uint32_t r = (uint32_t)((sinv * rho) & (B - 1));
        TA aAr = 0, aAi = 0, aBr = 0, aBi = 0;
#pragma unroll 4
        for (uint64_t j = j0 + lane; j < j0 + per; j += lanes) {
            const uint64_t m = rho + j * B;
            const TIn xv = x[m];
            const uint64_t t = (sinv * m) & mask;
            const int64_t tA = t >= half ? (int64_t)t - (int64_t)n : (int64_t)t;
            const int64_t uA = tA - g.t0;
            if (uA < -1 || uA >= iw) continue;
            const int64_t uB = uA + 1;
            const TA gA = uA >= 0 ? G[uA] : (TA)0;
            const TA gB = uB < iw ? G[uB] : (TA)0;
            const cx<TA> mv = M[(tA - (int64_t)r) / iB - Llo];
            const TA xr = (TA)xv.x, xi = (TA)xv.y;
            const TA pr = mv.r * xr - mv.i * xi;
            const TA pi = mv.r * xi + mv.i * xr;
            aAr += gA * pr;
            aAi += gA * pi;
            aBr += gB * pr;
            aBi += gB * pi;
        }
        VA[lane * B + r] = cx<TA>{aAr, aAi};
        VB[lane * B + r] = cx<TA>{aBr, aBi};
    }
    __syncthreads();
    double* out = A.partial + ((uint64_t)job * A.parts + part) * 4 * (uint64_t)A.Bmax;
    for (uint32_t r = threadIdx.x; r < B; r += kThreads) {
        cx<TA> sa = VA[r], sb = VB[r];
        for (uint32_t l = 1; l < lanes; ++l) {
            sa = cadd(sa, VA[l * B + r]);
            sb = cadd(sb, VB[l * B + r]);
        }
        out[2 * r] = (double)sa.r;
        out[2 * r + 1] = (double)sa.i;
        out[2 * B + 2 * r] = (double)sb.r;
        out[2 * B + 2 * r + 1] = (double)sb.i;
    }
}

// Stage 2: one workgroup per job sums its partials in part order, applies
// the modulation, runs the FFT and stores the job's raw bins.
template <class TA>
__global__ void __launch_bounds__(kThreads) k_h2b_rsplit(H2BArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t job = blockIdx.x;
    SplitJob J;
    if (!split_job(A, job, J)) return;
    const RoundDev g = A.geom[J.r];
    const uint32_t B = g.B;
    cx<TA>* VA = reinterpret_cast<cx<TA>*>(smem);
    cx<TA>* VB = VA + B;
    const auto* tw = reinterpret_cast<const typename TwTraits<TA>::V*>(A.tw);
    const double* base = A.partial + (uint64_t)job * A.parts * 4 * (uint64_t)A.Bmax;
    for (uint32_t r = threadIdx.x; r < B; r += kThreads) {
        double ar = 0, ai = 0, br = 0, bi = 0;
        for (uint32_t p = 0; p < A.parts; ++p) {
            const double* q = base + (uint64_t)p * 4 * A.Bmax;
            ar += q[2 * r];
            ai += q[2 * r + 1];
            br += q[2 * B + 2 * r];
            bi += q[2 * B + 2 * r + 1];
        }
        VA[r] = cx<TA>{(TA)ar, (TA)ai};
        VB[r] = cx<TA>{(TA)br, (TA)bi};
    }
    __syncthreads();
    finalize_folds<TA, kThreads>(VA, VB, A.n, J.sigma, J.b, 1, B, 1);
    __syncthreads();
    lds_fft2<TA, kThreads>(VA, VB, B, A.Bmax, tw);
    double* out0 = A.raw + (((uint64_t)J.sig * A.raw_rounds + J.r) * A.nhash) * (uint64_t)A.Bmax * 2;
    store_bins<TA, kThreads>(VA, VB, B, g.logB, A.Bmax, 1, tw, A.sqrt_n, out0, out0 + 2 * (uint64_t)A.Bmax);
}

// ------------------------------------------------------------------ launch --
bool h2b_threads_ok(uint32_t threads) { return threads == 256 || threads == 512 || threads == 1024; }

// The Kaiser window's G' table (plan time): one workgroup per frequency f
// (grid-stride) sums the window's response at f in FP64, each thread a
// strided share of the samples with the phase from the exact integer
// (f t) mod n, then a fixed-order tree in LDS.
__global__ void __launch_bounds__(256) k_window_response(const double* __restrict__ G, uint64_t w, int64_t t0,
                                                         uint64_t n, uint64_t B, double alpha, double* out,
                                                         uint64_t count) {
    __shared__ double part[256];
    const uint32_t tid = threadIdx.x;
    const uint64_t mask = n - 1;
    for (uint64_t f = blockIdx.x; f < count; f += gridDim.x) {
        if ((double)(f * 2 * B) <= (1.0 - alpha) * (double)n || f * 2 * B >= n) {
            if (tid == 0) out[f] = f * 2 * B >= n ? 0.0 : 1.0;
            continue;   // uniform over the workgroup
        }
        double acc = 0.0;
        for (uint64_t u = tid; u < w; u += 256) {
            const uint64_t m = (f * (uint64_t)(t0 + (int64_t)u)) & mask;
            acc += G[u] * cospi(2.0 * (double)m / (double)n);
        }
        part[tid] = acc;
        __syncthreads();
        for (uint32_t h = 128; h > 0; h >>= 1) {
            if (tid < h) part[tid] += part[tid + h];
            __syncthreads();
        }
        if (tid == 0) out[f] = fmin(1.0, fmax(0.0, part[0]));
        __syncthreads();
    }
}

hipError_t launch_window_response(const double* G, uint64_t w, int64_t t0, uint64_t n, uint32_t B, double alpha,
                                  double* out, uint64_t count, hipStream_t s) {
    const uint64_t blocks = count < 65536 ? count : 65536;
    hipLaunchKernelGGL(k_window_response, dim3((uint32_t)blocks), dim3(256), 0, s, G, w, t0, n, (uint64_t)B, alpha,
                       out, count);
    return hipGetLastError();
}

size_t h2b_pair_lds_bytes(uint32_t Bmax, uint64_t max_mcount, bool acc_f64, uint32_t threads, bool tri) {
    const size_t csz = acc_f64 ? 16 : 8;
    const size_t slots = Bmax >= threads ? Bmax : threads;
    return ((tri ? 4 : 2) * slots + max_mcount) * csz;
}

template <class TIn, class TA, uint32_t NT>
static hipError_t launch_pair_nt(const H2BArgs& a, uint32_t grid, hipStream_t s) {
    const bool tri = a.gamma != 0;
    const size_t lds = h2b_pair_lds_bytes(a.Bmax, a.mcap, sizeof(TA) == 8, NT, tri);
    hipError_t e = tri ? allow_lds(k_h2b_pair<TIn, TA, NT, true>, lds) : allow_lds(k_h2b_pair<TIn, TA, NT, false>, lds);
    if (e != hipSuccess) return e;
    if (tri) hipLaunchKernelGGL((k_h2b_pair<TIn, TA, NT, true>), dim3(grid), dim3(NT), lds, s, a);
    else hipLaunchKernelGGL((k_h2b_pair<TIn, TA, NT, false>), dim3(grid), dim3(NT), lds, s, a);
    return hipGetLastError();
}

// Workgroup size of the batched pair launch: a.threads (256, 512 or 1024;
// 0 = 256), chosen per plan.
template <class TIn, class TA>
static hipError_t launch_pair_t(const H2BArgs& a, uint32_t grid, hipStream_t s) {
    switch (a.threads) {
        case 512: return launch_pair_nt<TIn, TA, 512>(a, grid, s);
        case 1024: return launch_pair_nt<TIn, TA, 1024>(a, grid, s);
        case 0:
        case 256: return launch_pair_nt<TIn, TA, 256>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
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
    const uint32_t grid = a.explicit_job ? 1u : (a.jobs ? a.count * a.njobs : a.count * a.nrounds);
    if (in_c128) return acc_f64 ? launch_pair_t<double2, double>(a, grid, s) : launch_pair_t<double2, float>(a, grid, s);
    return acc_f64 ? launch_pair_t<float2, double>(a, grid, s) : launch_pair_t<float2, float>(a, grid, s);
}

hipError_t launch_h2b_split(const H2BArgs& a, uint32_t round, bool in_c128, bool acc_f64, hipStream_t s) {
    const size_t lds = h2b_pair_lds_bytes(a.Bmax, a.mcap, acc_f64, kThreads, false);
    if (in_c128) return acc_f64 ? launch_split_t<double2, double>(a, round, lds, s)
                                : launch_split_t<double2, float>(a, round, lds, s);
    return acc_f64 ? launch_split_t<float2, double>(a, round, lds, s) : launch_split_t<float2, float>(a, round, lds, s);
}

template <class TIn, class TA>
static hipError_t launch_psplit_t(const H2BArgs& a, uint32_t jobs, size_t lds, hipStream_t s) {
    hipError_t e = allow_lds(k_h2b_psplit<TIn, TA>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_h2b_psplit<TIn, TA>), dim3(a.parts, jobs), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_h2b_pair_split(const H2BArgs& a, bool in_c128, bool acc_f64, hipStream_t s) {
    const uint32_t jobs = a.count * a.nrounds;
    if (jobs == 0 || jobs > 65535 || a.parts < 2 || !a.partial) return hipErrorInvalidValue;
    const size_t lds = h2b_pair_lds_bytes(a.Bmax, a.mcap, acc_f64, kThreads, false);
    hipError_t e = in_c128 ? (acc_f64 ? launch_psplit_t<double2, double>(a, jobs, lds, s)
                                      : launch_psplit_t<double2, float>(a, jobs, lds, s))
                           : (acc_f64 ? launch_psplit_t<float2, double>(a, jobs, lds, s)
                                      : launch_psplit_t<float2, float>(a, jobs, lds, s));
    if (e != hipSuccess) return e;
    const size_t lds2 = 2 * (size_t)a.Bmax * (acc_f64 ? 16 : 8);
    e = acc_f64 ? allow_lds(k_h2b_rsplit<double>, lds2) : allow_lds(k_h2b_rsplit<float>, lds2);
    if (e != hipSuccess) return e;
    if (acc_f64) hipLaunchKernelGGL((k_h2b_rsplit<double>), dim3(jobs), dim3(kThreads), lds2, s, a);
    else hipLaunchKernelGGL((k_h2b_rsplit<float>), dim3(jobs), dim3(kThreads), lds2, s, a);
    return hipGetLastError();
}

template <class TIn, class TA>
static hipError_t launch_pstream_t(const H2BArgs& a, uint32_t jobs, size_t lds, hipStream_t s) {
    hipError_t e = allow_lds(k_h2b_pstream<TIn, TA>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_h2b_pstream<TIn, TA>), dim3(a.parts, jobs), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

size_t h2b_stream_lds_bytes(uint32_t Bmax, uint64_t max_mcount, bool acc_f64) {
    const size_t csz = acc_f64 ? 16 : 8;
    const size_t slots = Bmax >= kThreads ? Bmax : kThreads;
    return (2 * slots + max_mcount) * csz;
}

hipError_t launch_h2b_pair_stream(const H2BArgs& a, bool in_c128, bool acc_f64, hipStream_t s) {
    const uint32_t jobs = a.count * a.nrounds;
    if (jobs == 0 || jobs > 65535 || a.parts < 1 || !a.partial) return hipErrorInvalidValue;
    const size_t lds = h2b_stream_lds_bytes(a.Bmax, a.mcap, acc_f64);
    hipError_t e = in_c128 ? (acc_f64 ? launch_pstream_t<double2, double>(a, jobs, lds, s)
                                      : launch_pstream_t<double2, float>(a, jobs, lds, s))
                           : (acc_f64 ? launch_pstream_t<float2, double>(a, jobs, lds, s)
                                      : launch_pstream_t<float2, float>(a, jobs, lds, s));
    if (e != hipSuccess) return e;
    const size_t lds2 = 2 * (size_t)a.Bmax * (acc_f64 ? 16 : 8);
    e = acc_f64 ? allow_lds(k_h2b_rsplit<double>, lds2) : allow_lds(k_h2b_rsplit<float>, lds2);
    if (e != hipSuccess) return e;
    if (acc_f64) hipLaunchKernelGGL((k_h2b_rsplit<double>), dim3(jobs), dim3(kThreads), lds2, s, a);
    else hipLaunchKernelGGL((k_h2b_rsplit<float>), dim3(jobs), dim3(kThreads), lds2, s, a);
    return hipGetLastError();
}

hipError_t launch_h2b_reduce(const H2BArgs& a, uint32_t round, bool acc_f64, hipStream_t s) {
    const size_t lds = 2 * (size_t)a.Bmax * (acc_f64 ? 16 : 8);
    hipError_t e = acc_f64 ? allow_lds(k_h2b_reduce<double>, lds) : allow_lds(k_h2b_reduce<float>, lds);
    if (e != hipSuccess) return e;
    if (acc_f64) hipLaunchKernelGGL((k_h2b_reduce<double>), dim3(1), dim3(kThreads), lds, s, a, round);
    else hipLaunchKernelGGL((k_h2b_reduce<float>), dim3(1), dim3(kThreads), lds, s, a, round);
    return hipGetLastError();
}

}  // namespace sfft
