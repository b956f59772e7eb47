// Device building blocks of the HashToBins pair kernels (permuted gather,
// window x modulation, fold into B residues, B-point FFT in LDS, scaled
// store).
#pragma once
#include "sfft_device.hpp"

namespace sfft {

// Samples each thread keeps in flight in the gather loop.
#ifndef SFFT_GATHER_UNROLL
#define SFFT_GATHER_UNROLL 4
#endif
constexpr int kGatherUnroll = SFFT_GATHER_UNROLL;

// In-place radix-2 decimation-in-frequency FFT of VA and VB (B points each,
// natural-order input, bit-reversed output), unnormalised, sign -:
// X_j = sum_r V_r exp(-2 pi i j r / B).  tw holds exp(-2 pi i m / Bmax),
// m < Bmax.  Stages whose butterflies span 64 points or more go through LDS
// (one barrier each); from B = 64 on, the last six (span 32 .. 1) pair lanes
// of one wavefront: each wave takes 64-point blocks, one point per lane, and
// exchanges partners with shuffles.
template <class TA, uint32_t NT>
__device__ void lds_fft2(cx<TA>* VA, cx<TA>* VB, uint32_t B, uint32_t Bmax,
                         const typename TwTraits<TA>::V* tw) {
    const uint32_t tid = threadIdx.x;
    const uint32_t hb = B >> 1;
    const uint32_t lds_last = B >= 64 ? 64u : 1u;
    for (uint32_t half = hb; half >= lds_last; half >>= 1) {
        const uint32_t tstride = Bmax / (2 * half);
        for (uint32_t k = tid; k < B; k += NT) {
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
    if (B >= 64) {
        const uint32_t lane = tid & 63u, wave = tid >> 6;
        const uint32_t per = B >> 6;            // 64-point blocks per transform
        for (uint32_t blk = wave; blk < 2 * per; blk += NT / 64) {
            cx<TA>* V = blk < per ? VA : VB;
            const uint32_t at = ((blk < per ? blk : blk - per) << 6) + lane;
            cx<TA> v = V[at];
#pragma unroll
            for (uint32_t half = 32; half >= 1; half >>= 1) {
                const cx<TA> u{__shfl_xor(v.r, (int)half, 64), __shfl_xor(v.i, (int)half, 64)};
                const auto t = tw[(lane & (half - 1)) * (Bmax / (2 * half))];
                // the lower point of a pair keeps a + b, the upper (a - b) w^j
                v = (lane & half) ? cmul(csub(u, v), cx<TA>{t.x, t.y}) : cadd(v, u);
            }
            V[at] = v;
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
// are added into VA/VB[part * B + r].  UNROLL samples per thread are kept
// in flight.
//
// TRI adds a third hashing at shift a + gamma (gamma > beta, beta < w), with
// weight G_{t_A + gamma} into VC: for gamma < w + beta the samples t_A in
// [t0 - gamma, t0 + w) feed all three; a larger gamma reads its own window
// [t0 - gamma, t0 - gamma + w) beside the pair's [t0 - beta, t0 + w).
template <class TIn, class TA, uint32_t NT, bool TRI = false, int UNROLL = kGatherUnroll>
__device__ void accumulate_pair(const TIn* __restrict__ x, const TA* __restrict__ G, cx<TA>* VA,
                                cx<TA>* VB, cx<TA>* M, uint64_t n, uint64_t sigma, uint64_t a,
                                uint64_t beta, uint64_t b, uint32_t B, uint32_t logB, uint64_t w,
                                int64_t t0, int64_t Lwin_lo, int64_t Lwin_hi, uint32_t parts,
                                cx<TA>* VC = nullptr, uint64_t gamma = 0) {
    const uint32_t tid = threadIdx.x;
    const uint64_t mask = n - 1;
    const uint64_t c = (sigma * b) & mask;
    const uint64_t cB = (c * (uint64_t)B) & mask;
    const uint64_t sB = (sigma * (uint64_t)B) & mask;
    const int64_t iB = (int64_t)B;
    const int64_t iw = (int64_t)w;
    const int64_t ibeta = (int64_t)beta;
    const int64_t igamma = (int64_t)gamma;
    int64_t lo[2], hi[2];
    int nseg;
    if (TRI) {
        lo[0] = t0 - igamma;
        hi[0] = igamma < iw + ibeta ? t0 + iw : lo[0] + iw;
        lo[1] = t0 - ibeta;
        hi[1] = t0 + iw;
        nseg = igamma < iw + ibeta ? 1 : 2;
    } else if (beta < w) {
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
        for (int64_t L = Llo + tid; L <= Lhi; L += NT)
            M[L - Llo] = to_cx<TA>(omega_d((cB * (uint64_t)L) & mask, n));
        __syncthreads();
        for (uint32_t slot = tid; slot < parts * B; slot += NT) {
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
            TA aAr = 0, aAi = 0, aBr = 0, aBi = 0, aCr = 0, aCi = 0;
            const cx<TA>* Mp = M + (L0 - Llo);
            const int64_t cnt = L1 - L0 + 1;
#pragma unroll UNROLL
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
                if (TRI) {
                    const int64_t uC = uA + igamma;
                    const bool inC = (uC >= 0) & (uC < iw);
                    const TA gC = inC ? G[inC ? uC : 0] : (TA)0;
                    aCr += gC * pr;
                    aCi += gC * pi;
                }
                idx = (idx + sB) & mask;
                tA += iB;
            }
            VA[slot] = cadd(VA[slot], cx<TA>{aAr, aAi});
            VB[slot] = cadd(VB[slot], cx<TA>{aBr, aBi});
            if (TRI) VC[slot] = cadd(VC[slot], cx<TA>{aCr, aCi});
        }
    }
}

// Sum the parts of column r, apply omega^{c r} (hashing A) and
// omega^{c (r + beta)} (hashing B), leaving natural-order folds in VA/VB[0, B).
template <class TA, uint32_t NT>
__device__ void finalize_folds(cx<TA>* VA, cx<TA>* VB, uint64_t n, uint64_t sigma, uint64_t b,
                               uint64_t beta, uint32_t B, uint32_t parts) {
    const uint64_t mask = n - 1;
    const uint64_t c = (sigma * b) & mask;
    for (uint32_t r = threadIdx.x; r < B; r += NT) {
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
// out0 == nullptr stores hashing B only.
template <class TA, uint32_t NT>
__device__ void store_bins(const cx<TA>* VA, const cx<TA>* VB, uint32_t B, uint32_t logB, uint32_t Bmax,
                           uint64_t beta, const typename TwTraits<TA>::V* tw, double sqrt_n,
                           double* out0, double* out1) {
    const uint32_t bstride = Bmax / B;
    for (uint32_t j = threadIdx.x; j < B; j += NT) {
        const uint32_t br = bitrev(j, logB);
        const cx<TA> va = VA[br];
        cx<TA> vb = VB[br];
        const uint32_t e = (uint32_t)(((uint64_t)j * (beta & (B - 1))) & (B - 1));
        const auto t = tw[e * bstride];
        vb = cmul(vb, cx<TA>{t.x, t.y});
        if (out0) {
            out0[2 * j] = (double)va.r * sqrt_n;
            out0[2 * j + 1] = (double)va.i * sqrt_n;
        }
        out1[2 * j] = (double)vb.r * sqrt_n;
        out1[2 * j + 1] = (double)vb.i * sqrt_n;
    }
}

}  // namespace sfft
