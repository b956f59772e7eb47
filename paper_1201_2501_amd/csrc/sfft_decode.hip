// Decoders of the sparse FFT for gfx950: exact mode (Algorithm 1,
// NoiselessSparseFFT) and general mode (Algorithms 2 and 3, SparseFFT with
// LocateSignal/LocateInner and EstimateValues), each followed by the FP64
// median re-estimation of the recovered coefficients and the output.
//
// One workgroup per signal walks the rounds on raw bins computed up front
// (HashToBins steps 1-3 do not depend on zhat).  zhat is a sorted index list
// with values in HBM, double buffered.  Every per-round grouping of zhat
// entries by bin is an LDS counting sort (atomic counts, block scan,
// scatter, insertion sort inside each bin by entry), so the subtraction of
// HashToBins step 4 runs per bin in ascending index order - a fixed order,
// without float atomics.  Candidates are compacted before they are sorted,
// and zhat merges use binary search in LDS plus one block scan.
#include "sfft_device.hpp"

namespace sfft {

namespace {

constexpr uint64_t kNone = ~0ull;
constexpr uint32_t kCandShift = 13;                        // candidate key: index << 13 | slot
constexpr uint64_t kSlotMask = (1ull << kCandShift) - 1;
constexpr uint64_t kFound = 1ull << 63;
constexpr uint32_t kMaxMeas = 64;                          // medians over at most 64 values
// Threads per signal.  The decode is a chain of short dependent steps; a
// block of several waves spreads each step's bins and entries over more
// SIMDs and hides the latency of one wave behind the others.
#ifndef SFFT_DECODE_THREADS
#define SFFT_DECODE_THREADS 256
#endif
constexpr uint32_t kDec = SFFT_DECODE_THREADS;
static_assert(kDec % 64 == 0 && kDec <= 1024, "decode blocks are whole waves");
constexpr uint32_t kUnroll = 4;                            // bins/entries per lane with loads in flight together
constexpr size_t kLdsLimit = 160 * 1024;                  // per CU
constexpr size_t kLdsTarget = kLdsLimit / 2;               // optional parts keep two decode blocks per CU

}  // namespace

// ------------------------------------------------------------- LDS layout --
struct DecodeLds {
    uint64_t* zl;      // [capz]      indices of the current zhat buffer
    uint64_t* zl2;     // [capz]      the next zhat indices, written by a merge (nullptr: restage from HBM)
    uint16_t* hk;      // [capz]      bin of each zhat entry under the current hashing (B <= 4096)
    uint16_t* ent;     // [capz]      zhat entries grouped by bin, ascending within a bin (capz <= 4096)
    uint32_t* first;   // [Bmax + 1]  first grouped position of each bin
    uint32_t* cnt;     // [Bmax]      bin counters (shares storage with nkey)
    uint64_t* ckey;    // [NK]        sort space
    uint64_t* nkey;    // [NK]        new zhat keys of a merge (shares storage with cnt)
    uint32_t* scan;    // [kDec / 64]
    uint32_t* misc;    // [8]
    uint32_t* sw;      // [kStateWords] the signal's decode state while a kernel runs
    cx<double>* t;     // [capz][2]   per-entry terms of one hashing (LDS, or HBM when they do not fit)
    uint32_t* ec;      // [capz]      re-estimation sample counts (LDS, or HBM when they do not fit)
    double* gp;        // [capz]      G'_{-o(i)} of each entry (per-round re-estimation)
};

// LDS work lists of the passes after the first.  A slot per entry not alone
// in any valid measurement (unresolved after pass 1), a task per (such
// entry, shared valid measurement) holding the task's sample with the
// neighbours pass 1 resolved already subtracted, and per task its
// neighbours still unresolved (their slot and the ratio c_m(e') / c_m(e)).
// The lists are read from HBM once; the passes then work in LDS, and an
// entry's value goes to HBM when it resolves.  Capacities are fixed; a
// signal that exceeds one takes the direct path (peel_direct), with the
// same results up to rounding.  The neighbour lists share kPeelNbBytes:
// exact mode's term coefficients are real (G'), so its ratios are too and
// take 8 bytes, general mode's 16.
constexpr uint32_t kPeelU = 192, kPeelT = 1536;
constexpr uint32_t kPeelNbBytes = 31040;
constexpr uint32_t kPeelNbReal = kPeelNbBytes / (8 + 2), kPeelNbCx = kPeelNbBytes / (16 + 2);
constexpr uint16_t kNoSlot = 0xFFFFu;
struct PeelScratch {
    uint64_t* crowd;   // [kPeelU]  shared valid measurements of the slot's entry
    uint64_t* ready;   // [kPeelU]  its tasks whose neighbours are all resolved (this pass)
    double2* zvu;      // [kPeelU]  its decoded value
    double2* delta;    // [kPeelU]  resolved value - decoded value
    uint64_t* task;    // [kPeelT]  slot | measurement << 16 | neighbours << 24 | first neighbour << 32
    double2* tsamp;    // [kPeelT]  the task's sample
    double* ratio;     // [nbcap]   c_m(e') / c_m(e) of each listed neighbour (re, or re and im)
    uint16_t* nbslot;  // [nbcap]   its slot (kNoSlot: it never resolves)
    uint16_t* ulist;   // [kPeelU]  entry of each slot
    uint16_t* tfirst;  // [kPeelU]  first task of each slot
    uint8_t* ustate;   // [kPeelU]  0 unresolved, 1 resolved, 2 resolved this pass
    uint32_t* cnt;     // [4]       slots, tasks, neighbours, overflow
    uint32_t nbcap;    // neighbour list capacity
    uint32_t real;     // real ratios (exact mode)
};

__host__ __device__ constexpr size_t peel_scratch_bytes() {
    return (size_t)kPeelU * (8 + 8 + 16 + 16 + 2 + 2 + 1) + (size_t)kPeelT * (8 + 16) + kPeelNbBytes + 16 + 16;
}

// Optional LDS parts, placed in this order while they fit.
enum : uint32_t { LDS_TERMS = 1, LDS_ZL2 = 2, LDS_EC = 4 };

__host__ __device__ inline uint32_t pow2_ceil_u32(uint32_t v) {
    uint32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// Bytes of the decode kernels' dynamic LDS with the optional parts `parts`;
// fills *L when base is given (absent parts left nullptr).
__host__ __device__ inline size_t decode_lds_layout(uint32_t capz, uint32_t Bmax, unsigned char* base, DecodeLds* L,
                                                    uint32_t parts) {
    const uint32_t NK = pow2_ceil_u32(capz > Bmax ? capz : Bmax);
    size_t off = 0;
    const size_t o_zl = off;
    off = align16(off + (size_t)capz * 8);
    const size_t o_hk = off;
    off = align16(off + (size_t)capz * 2);
    const size_t o_ent = off;
    off = align16(off + (size_t)capz * 2);
    const size_t o_first = off;
    off = align16(off + ((size_t)Bmax + 1) * 4);
    const size_t o_ckey = off;
    off = align16(off + (size_t)NK * 8);
    const size_t o_union = off;
    const size_t ubytes = (size_t)NK * 8 > (size_t)Bmax * 4 ? (size_t)NK * 8 : (size_t)Bmax * 4;
    off = align16(off + ubytes);
    const size_t o_scan = off;
    off = align16(off + (kDec / 64) * 4);
    const size_t o_misc = off;
    off = align16(off + 8 * 4);
    const size_t o_sw = off;
    off = align16(off + kStateWords * 4);
    const size_t o_t = off;
    if (parts & LDS_TERMS) off = align16(off + (size_t)capz * 32);
    const size_t o_zl2 = off;
    if (parts & LDS_ZL2) off = align16(off + (size_t)capz * 8);
    const size_t o_ec = off;
    if (parts & LDS_EC) off = align16(off + (size_t)capz * 4);
    if (base) {
        L->zl = reinterpret_cast<uint64_t*>(base + o_zl);
        L->hk = reinterpret_cast<uint16_t*>(base + o_hk);
        L->ent = reinterpret_cast<uint16_t*>(base + o_ent);
        L->first = reinterpret_cast<uint32_t*>(base + o_first);
        L->ckey = reinterpret_cast<uint64_t*>(base + o_ckey);
        L->cnt = reinterpret_cast<uint32_t*>(base + o_union);
        L->nkey = reinterpret_cast<uint64_t*>(base + o_union);
        L->scan = reinterpret_cast<uint32_t*>(base + o_scan);
        L->misc = reinterpret_cast<uint32_t*>(base + o_misc);
        L->sw = reinterpret_cast<uint32_t*>(base + o_sw);
        L->t = (parts & LDS_TERMS) ? reinterpret_cast<cx<double>*>(base + o_t) : nullptr;
        L->zl2 = (parts & LDS_ZL2) ? reinterpret_cast<uint64_t*>(base + o_zl2) : nullptr;
        L->ec = (parts & LDS_EC) ? reinterpret_cast<uint32_t*>(base + o_ec) : nullptr;
    }
    return off;
}

// The optional parts placed in LDS, in priority order, while two blocks
// still fit on a CU (512 signals resident at once on 256 CUs).
__host__ __device__ inline uint32_t decode_lds_parts(uint32_t capz, uint32_t Bmax) {
    uint32_t parts = 0;
    for (uint32_t p : {(uint32_t)LDS_TERMS, (uint32_t)LDS_ZL2, (uint32_t)LDS_EC})
        if (decode_lds_layout(capz, Bmax, nullptr, nullptr, parts | p) <= kLdsTarget) parts |= p;
    return parts;
}

size_t decode_lds_bytes(uint32_t capz, uint32_t Bmax) {
    return decode_lds_layout(capz, Bmax, nullptr, nullptr, decode_lds_parts(capz, Bmax));
}

// Lays out the dynamic LDS of one decode block.  Terms that do not fit go
// to the signal's HBM scratch `spill` ([capz][2] complex), sample counts to
// `ec_spill` ([capz]).
__device__ __forceinline__ DecodeLds decode_lds(unsigned char* smem, uint32_t capz, uint32_t Bmax, double* spill,
                                                uint32_t* ec_spill) {
    DecodeLds L;
    decode_lds_layout(capz, Bmax, smem, &L, decode_lds_parts(capz, Bmax));
    if (!L.t) L.t = reinterpret_cast<cx<double>*>(spill);
    if (!L.ec) L.ec = ec_spill;
    return L;
}

// Dynamic LDS of one per-round re-estimation block (exact mode): the bins
// of the entries, their grouping by bin and one term G' zhat per entry; the
// bin counters and the placement targets of group_by_bin share storage.
__host__ __device__ inline size_t reest_lds_layout(uint32_t capz, uint32_t Bmax, unsigned char* base, DecodeLds* L) {
    size_t off = 0;
    const size_t o_hk = off;
    off = align16(off + (size_t)capz * 2);
    const size_t o_ent = off;
    off = align16(off + (size_t)capz * 2);
    const size_t o_first = off;
    off = align16(off + ((size_t)Bmax + 1) * 4);
    const size_t o_union = off;
    off = align16(off + (size_t)(capz > Bmax ? capz : Bmax) * 4);
    const size_t o_scan = off;
    off = align16(off + (kDec / 64) * 4);
    const size_t o_t = off;
    off = align16(off + (size_t)capz * 16);
    const size_t o_gp = off;
    off = align16(off + (size_t)capz * 8);
    if (base) {
        *L = DecodeLds{};
        L->gp = reinterpret_cast<double*>(base + o_gp);
        L->hk = reinterpret_cast<uint16_t*>(base + o_hk);
        L->ent = reinterpret_cast<uint16_t*>(base + o_ent);
        L->first = reinterpret_cast<uint32_t*>(base + o_first);
        L->cnt = reinterpret_cast<uint32_t*>(base + o_union);
        L->ckey = reinterpret_cast<uint64_t*>(base + o_union);
        L->scan = reinterpret_cast<uint32_t*>(base + o_scan);
        L->t = reinterpret_cast<cx<double>*>(base + o_t);
    }
    return off;
}

size_t reest_lds_bytes(uint32_t capz, uint32_t Bmax) { return reest_lds_layout(capz, Bmax, nullptr, nullptr); }

// Dynamic LDS of the output kernels (k_exact_output, k_gen_output): zhat
// indices (general mode only: the exact kernel reads them from HBM), the
// resolution word of each entry (in hk), the state words and, at `peel`,
// the re-estimation's work lists (PeelScratch, peel_scratch_bytes() bytes),
// which the sort space of a truncated output overlays (it is used only
// after the values are resolved).
__host__ __device__ inline size_t output_lds_layout(uint32_t capz, uint32_t Bmax, bool with_zl, unsigned char* base,
                                                    DecodeLds* L, unsigned char** peel) {
    const uint32_t NK = pow2_ceil_u32(capz > Bmax ? capz : Bmax);
    size_t off = 0;
    const size_t o_zl = off;
    if (with_zl) off = align16(off + (size_t)capz * 8);
    const size_t o_hk = off;
    off = align16(off + (size_t)capz * 2);
    const size_t o_scan = off;
    off = align16(off + (kDec / 64) * 4);
    const size_t o_misc = off;
    off = align16(off + 8 * 4);
    const size_t o_sw = off;
    off = align16(off + kStateWords * 4);
    const size_t o_peel = off;
    const size_t pbytes = peel_scratch_bytes() > (size_t)NK * 8 ? peel_scratch_bytes() : (size_t)NK * 8;
    off = align16(off + pbytes);
    if (base) {
        *L = DecodeLds{};
        L->zl = with_zl ? reinterpret_cast<uint64_t*>(base + o_zl) : nullptr;
        L->hk = reinterpret_cast<uint16_t*>(base + o_hk);
        L->ckey = reinterpret_cast<uint64_t*>(base + o_peel);
        L->scan = reinterpret_cast<uint32_t*>(base + o_scan);
        L->misc = reinterpret_cast<uint32_t*>(base + o_misc);
        L->sw = reinterpret_cast<uint32_t*>(base + o_sw);
        *peel = base + o_peel;
    }
    return off;
}

size_t output_lds_bytes(uint32_t capz, uint32_t Bmax, bool with_zl) {
    return output_lds_layout(capz, Bmax, with_zl, nullptr, nullptr, nullptr);
}

// The signal's state words into LDS (start of a kernel) and back (end).
__device__ __forceinline__ void load_state(DecodeLds& L, const uint32_t* st) {
    if (threadIdx.x < kStateWords) L.sw[threadIdx.x] = st[threadIdx.x];
    __syncthreads();
}
__device__ __forceinline__ void store_state(const DecodeLds& L, uint32_t* st) {
    __syncthreads();
    if (threadIdx.x < kStateWords) st[threadIdx.x] = L.sw[threadIdx.x];
}

// Exclusive prefix sum of one value per thread of the block (kDec threads);
// returns the block total.  Wave scans by lane shuffles, then one pass over
// the per-wave totals.
__device__ uint32_t wave_block_scan(uint32_t v, uint32_t* scratch, uint32_t* out_prefix) {
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    uint32_t inc = v;
#pragma unroll
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    if constexpr (kDec == 64) {
        __syncthreads();
        *out_prefix = inc - v;
        return __shfl(inc, 63, 64);
    } else {
        __syncthreads();
        if (lane == 63) scratch[wave] = inc;
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (uint32_t w = 0; w < kDec / 64; ++w) {
            const uint32_t c = scratch[w];
            before += w < wave ? c : 0u;
            total += c;
        }
        *out_prefix = before + inc - v;
        return total;
    }
}

// Group entries e < zc by L.hk[e] < B: afterwards the entries of bin h are
// L.ent[L.first[h] .. L.first[h + 1]) in ascending order of e.
__device__ void group_by_bin(DecodeLds& L, uint32_t zc, uint32_t B) {
    const uint32_t tid = threadIdx.x;
    for (uint32_t h = tid; h < B; h += kDec) L.cnt[h] = 0;
    __syncthreads();
    for (uint32_t e = tid; e < zc; e += kDec) atomicAdd(&L.cnt[L.hk[e]], 1u);
    __syncthreads();
    const uint32_t per = (B + kDec - 1) / kDec;
    const uint32_t h0 = tid * per < B ? tid * per : B;
    const uint32_t h1 = h0 + per < B ? h0 + per : B;
    uint32_t local = 0;
    for (uint32_t h = h0; h < h1; ++h) local += L.cnt[h];
    uint32_t pre;
    wave_block_scan(local, L.scan, &pre);
    for (uint32_t h = h0; h < h1; ++h) {
        L.first[h] = pre;
        pre += L.cnt[h];
    }
    if (tid == 0) L.first[B] = zc;
    __syncthreads();
    for (uint32_t h = tid; h < B; h += kDec) L.cnt[h] = L.first[h];
    __syncthreads();
    for (uint32_t e = tid; e < zc; e += kDec) L.ent[atomicAdd(&L.cnt[L.hk[e]], 1u)] = (uint16_t)e;
    __syncthreads();
    // The atomic scatter leaves each bin in arbitrary order: every grouped
    // position ranks its entry within its bin's segment (entries are
    // distinct) and the entries are rewritten in ascending order.  The
    // targets pass through the candidate key space, idle while grouping.
    uint32_t* move = reinterpret_cast<uint32_t*>(L.ckey);
    for (uint32_t q = tid; q < zc; q += kDec) {
        const uint32_t v = L.ent[q];
        const uint32_t h = L.hk[v];
        const uint32_t p0 = L.first[h], p1 = L.first[h + 1];
        uint32_t rank = 0;
        for (uint32_t q2 = p0; q2 < p1; ++q2) rank += L.ent[q2] < v;
        move[q] = ((p0 + rank) << 16) | v;
    }
    __syncthreads();
    for (uint32_t q = tid; q < zc; q += kDec) {
        const uint32_t mv = move[q];
        L.ent[mv >> 16] = (uint16_t)(mv & 0xFFFFu);
    }
    __syncthreads();
}

__device__ __forceinline__ uint32_t lower_bound_lds(const uint64_t* a, uint32_t len, uint64_t v) {
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Ascending sort of the m distinct keys key[0, m) in LDS.  Up to one key
// per thread, each key's rank is counted against all others (broadcast LDS
// reads, two barriers); beyond that a bitonic network over the padded
// power of two.
__device__ void sort_unique_keys(uint64_t* key, uint32_t m) {
    const uint32_t tid = threadIdx.x;
    if (m <= kDec) {
        const uint64_t mine = tid < m ? key[tid] : 0;
        uint32_t rank = 0;
        if (tid < m) {
            // independent broadcast reads, eight in flight
            uint32_t q = 0;
            for (; q + 8 <= m; q += 8) {
                uint64_t k8[8];
#pragma unroll
                for (uint32_t u = 0; u < 8; ++u) k8[u] = key[q + u];
#pragma unroll
                for (uint32_t u = 0; u < 8; ++u) rank += k8[u] < mine ? 1u : 0u;
            }
            for (; q < m; ++q) rank += key[q] < mine ? 1u : 0u;
        }
        __syncthreads();
        if (tid < m) key[rank] = mine;
        __syncthreads();
        return;
    }
    const uint32_t NM = pow2_ceil_u32(m);
    for (uint32_t q = m + tid; q < NM; q += kDec) key[q] = kNone;
    bitonic_sort_u64<kDec>(key, NM);
}

// zhat += candidates.  L.ckey[0, m) holds keys index << 13 | slot (unsorted,
// unique indices) and cv[slot] the values.  Existing indices are updated in
// place; new ones are merged by index into the other zhat buffer, which
// becomes current.  Expects L.zl to hold the current indices.  Returns the
// number of new entries.
//
// kByBin (exact mode): the slot is the bin the candidate was decoded from and
// L.first/L.ent still group this round's entries by bin, so an existing
// entry with the candidate's index can only be in that bin; an update is
// marked in L.hk (0x8000 | slot; bins are below 0x8000) and applied by the
// entry's owner while copying.  The owners load the current values of their
// first kUnroll entries before the sort, so the copy does not wait on HBM.
// Otherwise a binary search finds existing entries, which are updated in
// HBM and read back by the copy.
template <bool kByBin>
__device__ uint32_t merge_candidates(DecodeLds& L, uint32_t m, const double* cv, uint64_t* zidx_all, double* zval_all,
                                     uint32_t sig, uint32_t capz) {
    const uint32_t tid = threadIdx.x;
    const uint32_t zc = L.sw[ST_ZCOUNT];
    const uint32_t zb = L.sw[ST_ZBUF];
    double* zv = zval_all + ((uint64_t)sig * 2 + zb) * capz * 2;
    double2 zcur[kUnroll];
    if constexpr (kByBin) {
        const double2* zv2 = reinterpret_cast<const double2*>(zv);
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u)
            if (tid + u * kDec < zc) zcur[u] = zv2[tid + u * kDec];
    }
    sort_unique_keys(L.ckey, m);
    const uint32_t per = (m + kDec - 1) / kDec;
    const uint32_t q0 = tid * per < m ? tid * per : m;
    const uint32_t q1 = q0 + per < m ? q0 + per : m;
    uint32_t fresh = 0;
    for (uint32_t q = q0; q < q1; ++q) {
        const uint64_t k = L.ckey[q];
        const uint64_t i = k >> kCandShift;
        const uint32_t j = (uint32_t)(k & kSlotMask);
        uint32_t e = zc;
        if constexpr (kByBin) {
            for (uint32_t p = L.first[j]; p < L.first[j + 1]; ++p)
                if (L.zl[L.ent[p]] == i) e = L.ent[p];
        } else {
            e = lower_bound_lds(L.zl, zc, i);
            if (e < zc && L.zl[e] != i) e = zc;
        }
        if (e < zc) {
            if constexpr (kByBin) {
                L.hk[e] = (uint16_t)(0x8000u | j);
            } else {
                zv[2 * e] += cv[2 * j];
                zv[2 * e + 1] += cv[2 * j + 1];
            }
            L.ckey[q] = k | kFound;
        } else {
            ++fresh;
        }
    }
    uint32_t pre;
    const uint32_t total = wave_block_scan(fresh, L.scan, &pre);
    for (uint32_t q = q0; q < q1; ++q)
        if (!(L.ckey[q] & kFound)) L.nkey[pre++] = L.ckey[q];
    __syncthreads();
    uint32_t mnew = total;
    if (zc + mnew > capz) {
        mnew = capz - zc;
        if (tid == 0) L.sw[ST_FLAGS] |= 2u;
    }
    uint64_t* zo = zidx_all + ((uint64_t)sig * 2 + (zb ^ 1)) * capz;
    double* zov = zval_all + ((uint64_t)sig * 2 + (zb ^ 1)) * capz * 2;
    uint64_t* zl2 = L.zl2;
    auto copy = [&](uint32_t e, double vr, double vi) {
        const uint64_t i = L.zl[e];
        uint32_t lo = 0, hi = mnew;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if ((L.nkey[mid] >> kCandShift) < i) lo = mid + 1; else hi = mid;
        }
        const uint32_t pos = e + lo;
        zo[pos] = i;
        if (zl2) zl2[pos] = i;
        if constexpr (kByBin) {
            const uint32_t mk = L.hk[e];
            if (mk & 0x8000u) {
                vr += cv[2 * (mk & 0x7FFFu)];
                vi += cv[2 * (mk & 0x7FFFu) + 1];
            }
        }
        zov[2 * pos] = vr;
        zov[2 * pos + 1] = vi;
    };
    if constexpr (kByBin) {
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
            const uint32_t e = tid + u * kDec;
            if (e < zc) copy(e, zcur[u].x, zcur[u].y);
        }
        for (uint32_t e = tid + kUnroll * kDec; e < zc; e += kDec) copy(e, zv[2 * e], zv[2 * e + 1]);
    } else {
        for (uint32_t e = tid; e < zc; e += kDec) copy(e, zv[2 * e], zv[2 * e + 1]);
    }
    for (uint32_t q = tid; q < mnew; q += kDec) {
        const uint64_t i = L.nkey[q] >> kCandShift;
        const uint32_t j = (uint32_t)(L.nkey[q] & kSlotMask);
        const uint32_t pos = q + lower_bound_lds(L.zl, zc, i);
        zo[pos] = i;
        if (zl2) zl2[pos] = i;
        zov[2 * pos] = cv[2 * j];
        zov[2 * pos + 1] = cv[2 * j + 1];
    }
    __syncthreads();
    if (tid == 0) {
        L.sw[ST_ZCOUNT] = zc + mnew;
        L.sw[ST_ZBUF] = zb ^ 1;
    }
    if (zl2) {
        L.zl2 = L.zl;
        L.zl = zl2;
    }
    __syncthreads();
    return mnew;
}

// Stage the current zhat indices (named by the LDS state words) into LDS;
// returns zc.
__device__ uint32_t stage_zhat(DecodeLds& L, const uint64_t* zidx_all, uint32_t sig, uint32_t capz) {
    const uint32_t zc = L.sw[ST_ZCOUNT];
    const uint64_t* zi = zidx_all + ((uint64_t)sig * 2 + L.sw[ST_ZBUF]) * capz;
    for (uint32_t e = threadIdx.x; e < zc; e += kDec) L.zl[e] = zi[e];
    __syncthreads();
    return zc;
}

// zc at the start of a round: L.zl is current when merges keep it in LDS,
// otherwise it is staged again.
__device__ __forceinline__ uint32_t round_zhat(DecodeLds& L, const uint64_t* zidx_all, uint32_t sig, uint32_t capz) {
    if (L.zl2) return L.sw[ST_ZCOUNT];
    return stage_zhat(L, zidx_all, sig, capz);
}

// Bins of every staged entry under (sigma, b, B), grouped.
__device__ void bin_zhat(DecodeLds& L, uint32_t zc, uint64_t sigma, uint64_t b, uint64_t n, uint32_t B) {
    for (uint32_t e = threadIdx.x; e < zc; e += kDec) L.hk[e] = (uint16_t)bin_offset(L.zl[e], sigma, b, n, B).h;
    __syncthreads();
    group_by_bin(L, zc, B);
}

// HashToBins step 4 for bin h: u_h - sum over the zhat entries of bin h, in
// ascending index order, of G'_{-o(i)} zhat_i omega^{shift sigma i}.
__device__ cx<double> corrected_bin(const DecodeLds& L, const double* rawv, uint32_t h, uint64_t shift,
                                    const double* zv, uint64_t sigma, uint64_t b, uint64_t n, uint32_t B,
                                    const WindowShape& ws) {
    cx<double> u{rawv[2 * h], rawv[2 * h + 1]};
    const uint64_t mask = n - 1;
    const uint64_t as = (shift * sigma) & mask;
    for (uint32_t q = L.first[h]; q < L.first[h + 1]; ++q) {
        const uint32_t e = L.ent[q];
        const uint64_t i = L.zl[e];
        const double gp = gprime(-bin_offset(i, sigma, b, n, B).o, n, B, ws);
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

// Median of the c <= K values src[q * 2] (q < c) by a bitonic network on
// registers; slots q >= c hold +inf and sort last.  An even count averages
// the two middle values.
template <uint32_t K>
__device__ __forceinline__ double median_net(const double* src, uint32_t c) {
    double a[K];
#pragma unroll
    for (uint32_t q = 0; q < K; ++q) a[q] = q < c ? src[2 * q] : __builtin_huge_val();
#pragma unroll
    for (uint32_t k = 2; k <= K; k <<= 1) {
#pragma unroll
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (uint32_t i = 0; i < K; ++i) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const double lo = fmin(a[i], a[l]), hi = fmax(a[i], a[l]);
                    const bool up = (i & k) == 0;
                    a[i] = up ? lo : hi;
                    a[l] = up ? hi : lo;
                }
            }
        }
    }
    double m0 = 0.0, m1 = 0.0;
#pragma unroll
    for (uint32_t q = 0; q < K; ++q) {
        if (q + 1 == c / 2) m0 = a[q];
        if (q == c / 2) m1 = a[q];
    }
    return (c & 1) ? m1 : 0.5 * (m0 + m1);
}

// The 64-value network holds 128 VGPRs per part: kept out of line so that
// its register demand stays out of the callers.
__device__ __noinline__ cx<double> median_cx64(const double* src, uint32_t c) {
    return {median_net<64>(src, c), median_net<64>(src + 1, c)};
}

// Median of c <= KMAX complex samples stored as (re, im) pairs, real and
// imaginary parts separately.
template <uint32_t KMAX>
__device__ cx<double> median_cx(const double* src, uint32_t c) {
    static_assert(KMAX == 32 || KMAX == 64, "median bound");
    if (c <= 8) return {median_net<8>(src, c), median_net<8>(src + 1, c)};
    if (c <= 16) return {median_net<16>(src, c), median_net<16>(src + 1, c)};
    if (KMAX == 32 || c <= 32) return {median_net<32>(src, c), median_net<32>(src + 1, c)};
    return median_cx64(src, c);
}

// Median of the samples src[m * stride] for the measurements m set in
// `mask` (popcount <= K), by the network of median_net.
template <uint32_t K>
__device__ __forceinline__ double median_net_mask(const double* src, uint64_t mask, uint64_t stride) {
    double a[K];
    const uint32_t c = __popcll(mask);
    uint64_t m = mask;
#pragma unroll
    for (uint32_t q = 0; q < K; ++q) {
        a[q] = __builtin_huge_val();
        if (m) {
            a[q] = src[(uint64_t)__builtin_ctzll(m) * stride];
            m &= m - 1;
        }
    }
#pragma unroll
    for (uint32_t k = 2; k <= K; k <<= 1) {
#pragma unroll
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (uint32_t i = 0; i < K; ++i) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const double lo = fmin(a[i], a[l]), hi = fmax(a[i], a[l]);
                    const bool up = (i & k) == 0;
                    a[i] = up ? lo : hi;
                    a[l] = up ? hi : lo;
                }
            }
        }
    }
    double m0 = 0.0, m1 = 0.0;
#pragma unroll
    for (uint32_t q = 0; q < K; ++q) {
        if (q + 1 == c / 2) m0 = a[q];
        if (q == c / 2) m1 = a[q];
    }
    return (c & 1) ? m1 : 0.5 * (m0 + m1);
}

// Complex median over the measurements in `mask` (at most KMAX: 32 or 64)
// of samples stored as (re, im) pairs `stride` doubles apart per
// measurement.  Out of line, so that the networks' registers do not add to
// the callers'.
template <uint32_t KMAX>
__device__ __noinline__ cx<double> median_cx_mask(const double* src, uint64_t mask, uint64_t stride) {
    static_assert(KMAX == 32 || KMAX == 64, "median bound");
    const uint32_t c = __popcll(mask);
    if (c <= 8) return {median_net_mask<8>(src, mask, stride), median_net_mask<8>(src + 1, mask, stride)};
    if (c <= 16) return {median_net_mask<16>(src, mask, stride), median_net_mask<16>(src + 1, mask, stride)};
    if (KMAX == 32 || c <= 32)
        return {median_net_mask<32>(src, mask, stride), median_net_mask<32>(src + 1, mask, stride)};
    return {median_net_mask<64>(src, mask, stride), median_net_mask<64>(src + 1, mask, stride)};
}

// Sort key ordering by |v| descending, then slot ascending (51 magnitude bits).
__device__ __forceinline__ uint64_t mag_key(double vr, double vi, uint32_t slot) {
    const double mg = sqrt(vr * vr + vi * vi);
    const uint64_t mb = (uint64_t)__double_as_longlong(mg) >> 12;
    return ((~mb & ((1ull << 51) - 1)) << 13) | slot;
}

// Write the output of one signal from re-estimated values fin[e] (e < zc,
// ascending index): all of them when keep_all, else those with
// |v| > half_theta; at most cap by (|v| desc, index asc); ascending index.
__device__ uint32_t write_output(DecodeLds& L, const uint64_t* zi, const double* fin, uint32_t zc, bool keep_all,
                                 double half_theta, uint32_t cap, double scale, uint64_t* oidx, double* oval,
                                 uint32_t* flags) {
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (zc + kDec - 1) / kDec;
    const uint32_t e0 = tid * per < zc ? tid * per : zc;
    const uint32_t e1 = e0 + per < zc ? e0 + per : zc;
    uint32_t cnt = 0;
    for (uint32_t e = e0; e < e1; ++e)
        cnt += keep_all || sqrt(fin[2 * e] * fin[2 * e] + fin[2 * e + 1] * fin[2 * e + 1]) > half_theta;
    uint32_t pre;
    const uint32_t nsurv = wave_block_scan(cnt, L.scan, &pre);
    uint32_t nout;
    if (nsurv <= cap) {
        for (uint32_t e = e0; e < e1; ++e) {
            const double vr = fin[2 * e], vi = fin[2 * e + 1];
            if (keep_all || sqrt(vr * vr + vi * vi) > half_theta) {
                oidx[pre] = zi[e];
                oval[2 * pre] = vr * scale;
                oval[2 * pre + 1] = vi * scale;
                ++pre;
            }
        }
        nout = nsurv;
    } else {
        *flags |= 1u;
        const uint32_t N = pow2_ceil_u32(zc);
        for (uint32_t e = tid; e < N; e += kDec) {
            bool keep = false;
            if (e < zc) keep = keep_all || sqrt(fin[2 * e] * fin[2 * e] + fin[2 * e + 1] * fin[2 * e + 1]) > half_theta;
            L.ckey[e] = keep ? mag_key(fin[2 * e], fin[2 * e + 1], e) : kNone;
        }
        bitonic_sort_u64<kDec>(L.ckey, N);
        for (uint32_t q = tid; q < N; q += kDec) L.ckey[q] = q < cap ? (L.ckey[q] & kSlotMask) : kNone;
        bitonic_sort_u64<kDec>(L.ckey, N);
        for (uint32_t q = tid; q < cap; q += kDec) {
            const uint32_t e = (uint32_t)L.ckey[q];
            oidx[q] = zi[e];
            oval[2 * q] = fin[2 * e] * scale;
            oval[2 * q + 1] = fin[2 * e + 1] * scale;
        }
        nout = cap;
    }
    __syncthreads();
    for (uint32_t q = nout + tid; q < cap; q += kDec) {
        oidx[q] = 0;
        oval[2 * q] = 0.0;
        oval[2 * q + 1] = 0.0;
    }
    return nout;
}

// ----------------------------------------------- final re-estimation --
// Samples of one signal's final re-estimation.  Measurement m is a decoded
// round (exact mode) or an EstimateValues hashing (general mode); for zhat
// entry e, slot s = m * ms + e * es holds
//   est[s]   (u_m[h] - sum over the other entries of the bin of c_m(e') zhat_e') / c_m(e),
//            complex, with the decoded zhat values
//   flag[s]  0 when G'_{-o_m(e)} < g_min, 1 when e is the only entry of its
//            bin, 2 when it shares the bin
//   grp[s]   first grouped position << 16 | member count of e's bin
//   coef[s]  c_m(e) = G'_{-o_m(e)} omega^{a sigma i_e}, the term entry e adds
//            to its bin (HashToBins lemma)
// (grp and coef written only for entries of shared bins), and
// ord[m * capz + q] lists measurement m's entries grouped by bin.
struct PeelView {
    double* est;
    const uint8_t* flag;
    const uint32_t* grp;
    const uint16_t* ord;
    const double* coef;
    uint64_t ms, es;   // slot strides
    uint32_t capz;
    uint32_t nmeas;    // measurements in use (<= 64)
};

constexpr uint32_t kMaxPasses = 8;

// real: exact mode (real term coefficients).
__device__ __forceinline__ PeelScratch peel_scratch(unsigned char* base, bool real) {
    PeelScratch P;
    P.real = real;
    P.nbcap = real ? kPeelNbReal : kPeelNbCx;
    P.zvu = reinterpret_cast<double2*>(base);
    P.delta = P.zvu + kPeelU;
    P.tsamp = P.delta + kPeelU;
    P.ratio = reinterpret_cast<double*>(P.tsamp + kPeelT);
    P.crowd = reinterpret_cast<uint64_t*>(P.ratio + P.nbcap * (real ? 1u : 2u));
    P.ready = P.crowd + kPeelU;
    P.task = P.ready + kPeelU;
    P.nbslot = reinterpret_cast<uint16_t*>(P.task + kPeelT);
    P.ulist = P.nbslot + P.nbcap;
    P.tfirst = P.ulist + kPeelU;
    P.ustate = reinterpret_cast<uint8_t*>(P.tfirst + kPeelU);
    P.cnt = reinterpret_cast<uint32_t*>(base + ((reinterpret_cast<uintptr_t>(P.ustate + kPeelU) - reinterpret_cast<uintptr_t>(base) + 15) & ~(uintptr_t)15));
    return P;
}

__device__ __forceinline__ uint64_t peel_mask(const PeelView& V, uint32_t e, uint8_t want) {
    uint64_t m = 0;
    for (uint32_t q = 0; q < V.nmeas; ++q) m |= (uint64_t)(V.flag[q * V.ms + (uint64_t)e * V.es] == want) << q;
    return m;
}

// est(m, e) -= sum over the neighbours e' of c_m(e') (v_e' - zhat_e') / c_m(e),
// for the neighbours nb[0, c) that res marks resolved.
__device__ __forceinline__ void peel_correct(const PeelView& V, uint32_t e, uint32_t m, const uint16_t* nb,
                                             uint32_t c, const double* zv, const double* fin, const uint16_t* res) {
    cx<double> acc{0.0, 0.0};
    for (uint32_t q = 0; q < c; ++q) {
        const uint32_t e2 = nb[q];
        if (res[e2] != 1) continue;
        const uint64_t s2 = m * V.ms + (uint64_t)e2 * V.es;
        const cx<double> c2{V.coef[2 * s2], V.coef[2 * s2 + 1]};
        const cx<double> d{fin[2 * e2] - zv[2 * e2], fin[2 * e2 + 1] - zv[2 * e2 + 1]};
        acc = cadd(acc, cmul(c2, d));
    }
    const uint64_t s = m * V.ms + (uint64_t)e * V.es;
    const cx<double> ce{V.coef[2 * s], V.coef[2 * s + 1]};
    const double n2 = ce.r * ce.r + ce.i * ce.i;
    const cx<double> q = cmul(acc, cx<double>{ce.r / n2, -ce.i / n2});
    V.est[2 * s] -= q.r;
    V.est[2 * s + 1] -= q.i;
}

// The passes after the first without LDS work lists: each unresolved entry
// walks its bins in HBM every pass.
template <uint32_t KMAX>
__device__ void peel_direct(const PeelView& V, uint32_t zc, const double* zv, double* fin, uint16_t* res,
                            uint32_t* misc) {
    const uint32_t tid = threadIdx.x;
    const uint64_t sstride = 2 * V.ms;
    auto neighbours = [&](uint32_t e, uint32_t m, uint32_t* c) {
        const uint32_t w = V.grp[m * V.ms + (uint64_t)e * V.es];
        *c = w & 0xFFFFu;
        return V.ord + (uint64_t)m * V.capz + (w >> 16);
    };
    for (uint32_t pass = 2; pass <= kMaxPasses; ++pass) {
        if (tid == 0) *misc = 0;
        __syncthreads();
        uint32_t mine = 0;
        for (uint32_t e = tid; e < zc; e += kDec) {
            if (res[e] != 0) continue;
            uint64_t ready = 0;
            for (uint64_t m = peel_mask(V, e, 2); m; m &= m - 1) {
                const uint32_t q = __builtin_ctzll(m);
                uint32_t c;
                const uint16_t* o = neighbours(e, q, &c);
                bool ok = true;
                for (uint32_t j = 0; j < c; ++j) ok &= o[j] == e || res[o[j]] == 1;
                if (ok) ready |= 1ull << q;
            }
            if (!ready) continue;
            for (uint64_t m = ready; m; m &= m - 1) {
                const uint32_t q = __builtin_ctzll(m);
                uint32_t c;
                const uint16_t* o = neighbours(e, q, &c);
                peel_correct(V, e, q, o, c, zv, fin, res);   // e itself is unresolved: skipped
            }
            const cx<double> v = median_cx_mask<KMAX>(V.est + 2 * (uint64_t)e * V.es, ready, sstride);
            fin[2 * e] = v.r;
            fin[2 * e + 1] = v.i;
            res[e] = 2;   // resolved in this pass: not yet read as resolved
            ++mine;
        }
        if (mine) atomicAdd(misc, mine);
        __syncthreads();
        const uint32_t got = *misc;
        for (uint32_t e = tid; e < zc; e += kDec)
            if (res[e] == 2) res[e] = 1;
        __syncthreads();
        if (!got) break;
    }
    for (uint32_t e = tid; e < zc; e += kDec) {
        if (res[e] != 0) continue;
        const uint64_t crowd = peel_mask(V, e, 2);
        cx<double> v{zv[2 * e], zv[2 * e + 1]};
        if (crowd) {
            for (uint64_t m = crowd; m; m &= m - 1) {
                const uint32_t q = __builtin_ctzll(m);
                uint32_t c;
                const uint16_t* o = neighbours(e, q, &c);
                peel_correct(V, e, q, o, c, zv, fin, res);
            }
            v = median_cx_mask<KMAX>(V.est + 2 * (uint64_t)e * V.es, crowd, sstride);
        }
        fin[2 * e] = v.r;
        fin[2 * e + 1] = v.i;
    }
    __syncthreads();
}

// Final values fin[e] of the zhat entries e < zc (decoded values zv), resolved
// in passes: pass 1 takes the median over the measurements where an entry
// is alone in its bin; pass p takes, for an unresolved entry, the median over
// the valid measurements whose other bin members were resolved before pass
// p, with their resolved values subtracted in place of the decoded ones;
// passes end when one resolves nothing (at most kMaxPasses).  Entries left
// take the median over all valid measurements, subtracting resolved values
// where a neighbour has one; entries without a valid measurement keep the
// decoded value.  Samples of entries that resolve are rewritten in place.
// res: [capz] LDS words; misc: one LDS word; P: LDS work lists (or nullptr:
// the direct path).
// KMAX: the most measurements of one entry (32 or 64).
template <uint32_t KMAX>
__device__ void peel_values(const PeelView& V, uint32_t zc, const double* zv, double* fin, uint16_t* res,
                            uint32_t* misc, const PeelScratch* P) {
    const uint32_t tid = threadIdx.x;
    const uint64_t sstride = 2 * V.ms;
    if (P && tid < 4) P->cnt[tid] = 0;
    __syncthreads();
    // pass 1; entries left for later passes get a slot (res = 0x8000 | slot)
    for (uint32_t e = tid; e < zc; e += kDec) {
        uint64_t iso = 0, crowd = 0;
        for (uint32_t q = 0; q < V.nmeas; ++q) {
            const uint8_t f = V.flag[q * V.ms + (uint64_t)e * V.es];
            iso |= (uint64_t)(f == 1) << q;
            crowd |= (uint64_t)(f == 2) << q;
        }
        res[e] = iso ? 1 : 0;
        if (iso) {
            const cx<double> v = median_cx_mask<KMAX>(V.est + 2 * (uint64_t)e * V.es, iso, sstride);
            fin[2 * e] = v.r;
            fin[2 * e + 1] = v.i;
        } else {
            fin[2 * e] = zv[2 * e];
            fin[2 * e + 1] = zv[2 * e + 1];
            if (crowd && P) {
                const uint32_t u = atomicAdd(&P->cnt[0], 1u);
                if (u < kPeelU) {
                    P->ulist[u] = (uint16_t)e;
                    P->crowd[u] = crowd;
                    P->zvu[u] = make_double2(zv[2 * e], zv[2 * e + 1]);
                    P->delta[u] = make_double2(0.0, 0.0);
                    P->ustate[u] = 0;
                    res[e] = 0x8000u | u;
                }
            }
        }
    }
    __syncthreads();
    // back to plain resolution words, then the direct path
    auto give_up = [&]() {
        for (uint32_t e = tid; e < zc; e += kDec)
            if (res[e] & 0x8000u) res[e] = 0;
        __syncthreads();
        peel_direct<KMAX>(V, zc, zv, fin, res, misc);
    };
    if (!P) {
        peel_direct<KMAX>(V, zc, zv, fin, res, misc);
        return;
    }
    const uint32_t U = P->cnt[0];
    if (U > kPeelU) return give_up();
    // one task per (slot, shared valid measurement), a slot's tasks in a row
    for (uint32_t u = tid; u < U; u += kDec) {
        const uint64_t crowd = P->crowd[u];
        uint32_t t = atomicAdd(&P->cnt[1], (uint32_t)__popcll(crowd));
        P->tfirst[u] = (uint16_t)(t < kPeelT ? t : 0);
        for (uint64_t m = crowd; m; m &= m - 1, ++t)
            if (t < kPeelT) P->task[t] = (uint64_t)u | (uint64_t)__builtin_ctzll(m) << 16;
    }
    __syncthreads();
    const uint32_t T = P->cnt[1];
    if (T > kPeelT) return give_up();
    // each task's sample with the neighbours resolved in pass 1 subtracted
    // (their values are final), and its other neighbours listed: one walk
    // of the bin's members counts them and takes room in the neighbour
    // lists, a second (cached) walk fills it
    for (uint32_t t = tid; t < T; t += kDec) {
        const uint64_t tk = P->task[t];
        const uint32_t e = P->ulist[tk & 0xFFFFu], q = (uint32_t)(tk >> 16) & 0xFFu;
        const uint64_t s = q * V.ms + (uint64_t)e * V.es;
        const uint32_t w = V.grp[s];
        const double2 es = make_double2(V.est[2 * s], V.est[2 * s + 1]);
        const cx<double> ce{V.coef[2 * s], V.coef[2 * s + 1]};
        const uint16_t* o = V.ord + (uint64_t)q * V.capz + (w >> 16);
        const uint32_t nm = w & 0xFFFFu;
        uint32_t left = 0;
#pragma unroll 4
        for (uint32_t i = 0; i < nm; ++i) left += o[i] != e && res[o[i]] != 1;
        const uint32_t off = atomicAdd(&P->cnt[2], left);
        const bool fits = left <= 255 && off + left <= P->nbcap;
        if (!fits) P->cnt[3] = 1;
        P->task[t] = tk | (uint64_t)(left & 0xFFu) << 24 | (uint64_t)off << 32;
        const double n2 = ce.r * ce.r + ce.i * ce.i;
        const cx<double> inv{ce.r / n2, -ce.i / n2};
        cx<double> acc{0.0, 0.0};
        uint32_t j = off;
#pragma unroll 4
        for (uint32_t i = 0; i < nm; ++i) {
            const uint32_t e2 = o[i];
            if (e2 == e) continue;
            const uint64_t s2 = q * V.ms + (uint64_t)e2 * V.es;
            const cx<double> c2{V.coef[2 * s2], V.coef[2 * s2 + 1]};
            const uint16_t r2 = res[e2];
            if (r2 == 1) {
                acc = cadd(acc, cmul(c2, cx<double>{fin[2 * e2] - zv[2 * e2], fin[2 * e2 + 1] - zv[2 * e2 + 1]}));
            } else if (fits) {
                const cx<double> ra = cmul(c2, inv);
                if (P->real) {
                    P->ratio[j] = ra.r;
                } else {
                    P->ratio[2 * j] = ra.r;
                    P->ratio[2 * j + 1] = ra.i;
                }
                P->nbslot[j++] = (r2 & 0x8000u) ? (uint16_t)(r2 & 0x7FFFu) : kNoSlot;
            }
        }
        const cx<double> d = cmul(acc, inv);
        P->tsamp[t] = make_double2(es.x - d.r, es.y - d.i);
    }
    __syncthreads();
    if (P->cnt[3]) return give_up();
    const double* ts = reinterpret_cast<const double*>(P->tsamp);
    auto subtract_resolved = [&](uint32_t t, uint64_t tk) {
        const uint32_t c = (uint32_t)(tk >> 24) & 0xFFu, off = (uint32_t)(tk >> 32);
        double2 v = P->tsamp[t];
        for (uint32_t j = off; j < off + c; ++j) {
            const uint16_t u2 = P->nbslot[j];
            if (u2 == kNoSlot || P->ustate[u2] != 1) continue;
            const double2 d = P->delta[u2];
            const double rx = P->real ? P->ratio[j] : P->ratio[2 * j];
            const double ry = P->real ? 0.0 : P->ratio[2 * j + 1];
            v.x -= rx * d.x - ry * d.y;
            v.y -= rx * d.y + ry * d.x;
        }
        P->tsamp[t] = v;
    };
    for (uint32_t pass = 2; pass <= kMaxPasses; ++pass) {
        for (uint32_t u = tid; u < U; u += kDec) P->ready[u] = 0;
        if (tid == 0) *misc = 0;
        __syncthreads();
        for (uint32_t t = tid; t < T; t += kDec) {
            const uint64_t tk = P->task[t];
            const uint32_t u = (uint32_t)(tk & 0xFFFFu);
            if (P->ustate[u] != 0) continue;
            const uint32_t c = (uint32_t)(tk >> 24) & 0xFFu, off = (uint32_t)(tk >> 32);
            bool ok = true;
            for (uint32_t j = off; j < off + c; ++j) ok &= P->nbslot[j] != kNoSlot && P->ustate[P->nbslot[j]] == 1;
            if (ok) atomicOr(reinterpret_cast<unsigned long long*>(&P->ready[u]), 1ull << (t - P->tfirst[u]));
        }
        __syncthreads();
        for (uint32_t t = tid; t < T; t += kDec) {
            const uint64_t tk = P->task[t];
            const uint32_t u = (uint32_t)(tk & 0xFFFFu);
            if (P->ustate[u] == 0 && (P->ready[u] >> (t - P->tfirst[u]) & 1)) subtract_resolved(t, tk);
        }
        __syncthreads();
        uint32_t mine = 0;
        for (uint32_t u = tid; u < U; u += kDec) {
            const uint64_t ready = P->ready[u];
            if (P->ustate[u] != 0 || !ready) continue;
            const cx<double> v = median_cx_mask<KMAX>(ts + 2 * (uint64_t)P->tfirst[u], ready, 2);
            const uint32_t e = P->ulist[u];
            fin[2 * e] = v.r;
            fin[2 * e + 1] = v.i;
            P->delta[u] = make_double2(v.r - P->zvu[u].x, v.i - P->zvu[u].y);
            P->ustate[u] = 2;   // resolved in this pass: not yet read as resolved
            ++mine;
        }
        if (mine) atomicAdd(misc, mine);
        __syncthreads();
        const uint32_t got = *misc;
        for (uint32_t u = tid; u < U; u += kDec)
            if (P->ustate[u] == 2) P->ustate[u] = 1;
        __syncthreads();
        if (!got) break;
    }
    // entries left: every shared valid measurement, resolved neighbours subtracted
    for (uint32_t t = tid; t < T; t += kDec) {
        const uint64_t tk = P->task[t];
        if (P->ustate[tk & 0xFFFFu] == 0) subtract_resolved(t, tk);
    }
    __syncthreads();
    for (uint32_t u = tid; u < U; u += kDec) {
        if (P->ustate[u] != 0) continue;
        const uint32_t nt = (uint32_t)__popcll(P->crowd[u]);
        const uint64_t all = nt >= 64 ? ~0ull : (1ull << nt) - 1;
        const cx<double> v = median_cx_mask<KMAX>(ts + 2 * (uint64_t)P->tfirst[u], all, 2);
        const uint32_t e = P->ulist[u];
        fin[2 * e] = v.r;
        fin[2 * e + 1] = v.i;
    }
    __syncthreads();
}

// =================================================================== exact
__device__ __forceinline__ const double* raw_bins(const DecodeArgs& D, uint32_t sig, uint32_t r, uint32_t a) {
    return D.raw + (((uint64_t)sig * D.rounds + r) * D.nhash + a) * (uint64_t)D.Bmax * 2;
}

// Per-entry terms of HashToBins step 4 under (sigma, b, B): the bin hk[e]
// of every staged entry, t[2e] = G'_{-o(i)} zhat_i and t[2e+1] =
// t[2e] omega^{sigma i} (the same term under the hashing with a = 1); then
// the entries are grouped by bin.  zp holds zhat of this lane's first
// kUnroll entries (e = tid + u kDec), loaded ahead by the caller.
__device__ __forceinline__ void term_entry(DecodeLds& L, uint32_t e, double2 z, uint64_t sigma, uint64_t b,
                                           uint64_t n, uint32_t B, const WindowShape& ws) {
    const uint64_t i = L.zl[e];
    const BinOffset bo = bin_offset(i, sigma, b, n, B);
    L.hk[e] = (uint16_t)bo.h;
    // the phase factor first: its sincos overlaps the load of a tabulated G'
    const cx<double> om = omega_d((sigma * i) & (n - 1), n);
    const double gp = gprime(-bo.o, n, B, ws);
    const cx<double> c0{gp * z.x, gp * z.y};
    L.t[2 * e] = c0;
    L.t[2 * e + 1] = cmul(c0, om);
}

__device__ void stage_terms(DecodeLds& L, uint32_t zc, const double2 (&zp)[kUnroll], const double2* zv2,
                            uint64_t sigma, uint64_t b, uint64_t n, uint32_t B, const WindowShape& ws) {
    const uint32_t tid = threadIdx.x;
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; ++u) {
        const uint32_t e = tid + u * kDec;
        if (e < zc) term_entry(L, e, zp[u], sigma, b, n, B, ws);
    }
    for (uint32_t e = tid + kUnroll * kDec; e < zc; e += kDec) term_entry(L, e, zv2[e], sigma, b, n, B, ws);
    __syncthreads();
    group_by_bin(L, zc, B);
}

// Multi-shift refinement of a coarse permuted position p0 (the LocateInner
// idea of Algorithm 3 with one more hashing, at shift A = refine_shift):
// bin j of the hashing at shift A, less the zhat terms of the bin (each
// G'_{-o(i)} zhat_i omega^{A sigma i}, ascending index order), gives u_A;
// an isolated coefficient at permuted position p has u_A = u omega^{A p}.
// The position c in [p0 - E, p0 + E] whose angle 2 pi (A c mod n) / n is
// nearest (circularly) to the phase of u / u_A wins; ties keep the first
// (smallest) c.  Angles are exact in integers, so FP32 bins only need to
// resolve the spacing 2 pi A / n.
// With c = p0 - E + q, A c = base + A q (mod n) and A (2E + 1) < n, so A q
// runs once through [0, n) without wrapping: the circular distance to the
// target d0 = phase n / (2 pi) - base is smallest at q next to d0 / A or at
// q = 0 or 2E.  Those candidates (with one more on each side of d0 / A, for
// the rounding of d0) are scored in ascending q with the scan's formula;
// every other q is at least 2 pi A / n farther, so the winner is the scan's.
__device__ __noinline__ uint64_t refine_position(const DecodeArgs& D, const DecodeLds& L, uint32_t j, double u0r,
                                                 double u0i, double2 aA, uint64_t sigma, uint64_t n, uint64_t p0) {
    const double two_pi = 6.283185307179586;
    const uint64_t mask = n - 1, A = D.refine_shift, E = D.refine_window;
    double uAr = aA.x, uAi = aA.y;
    for (uint32_t q = L.first[j]; q < L.first[j + 1]; ++q) {
        const uint32_t e = L.ent[q];
        const uint64_t i = L.zl[e];
        const cx<double> cA = cmul(L.t[2 * e], omega_d((A * ((sigma * i) & mask)) & mask, n));
        uAr -= cA.r;
        uAi -= cA.i;
    }
    const double zr = u0r * uAr + u0i * uAi;
    const double zim = u0i * uAr - u0r * uAi;
    double ph = atan2(zim, zr);
    if (ph < 0.0) ph += two_pi;
    const uint64_t c0 = (p0 - E) & mask;
    double d0 = ph / two_pi * (double)n - (double)((A * c0) & mask);
    if (d0 < 0.0) d0 += (double)n;
    const int64_t qm = (int64_t)floor(d0 / (double)A);
    const int64_t top = (int64_t)(2 * E);
    const int64_t cand[6] = {0, qm - 1, qm, qm + 1, qm + 2, top};
    uint64_t best = p0;
    double bestd = INFINITY;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int64_t q = cand[k] < 0 ? 0 : (cand[k] > top ? top : cand[k]);
        const uint64_t c = (c0 + (uint64_t)q) & mask;
        const double ang = two_pi * (double)((A * c) & mask) / (double)n;
        double d = fabs(ang - ph);
        d = d < two_pi - d ? d : two_pi - d;
        if (d < bestd) {
            bestd = d;
            best = c;
        }
    }
    return best;
}

// Decode bin j of one round from its raw pair (u0, u1): subtract the zhat
// terms of the bin in ascending index order, then, when |u0| > theta, the
// phase of u1 / u0 names the frequency (refined by the hashing at shift
// refine_shift when the plan has one, rA its raw bins).  Returns whether
// |u0| > theta.  REF: the plan has the refinement hashing (a separate
// instantiation, so the plain decode keeps its registers).
template <bool REF>
__device__ __forceinline__ bool exact_bin(const DecodeArgs& D, DecodeLds& L, uint32_t j, double2 a0, double2 a1,
                                          uint64_t sigma, uint64_t sinv, uint64_t b, uint64_t n, uint32_t B,
                                          const WindowShape& ws, double* cv, const double2* rA) {
    const double two_pi = 6.283185307179586;
    const uint64_t mask = n - 1;
    double u0r = a0.x, u0i = a0.y, u1r = a1.x, u1i = a1.y;
    for (uint32_t q = L.first[j]; q < L.first[j + 1]; ++q) {
        const uint32_t e = L.ent[q];
        const cx<double> c0 = L.t[2 * e], c1 = L.t[2 * e + 1];
        u0r -= c0.r;
        u0i -= c0.i;
        u1r -= c1.r;
        u1i -= c1.i;
    }
    const double mag = sqrt(u0r * u0r + u0i * u0i);
    if (!(mag > D.theta)) return false;
    if (D.ratio_tol > 0.0) {
        // an isolated coefficient has equal magnitudes at both shifts
        const double m0 = u0r * u0r + u0i * u0i, m1 = u1r * u1r + u1i * u1i;
        if (fabs(m1 - m0) > D.ratio_tol * m0) return true;
    }
    const double zr = u0r * u1r + u0i * u1i;
    const double zim = u0i * u1r - u0r * u1i;
    double phi = atan2(zim, zr);
    if (phi < 0.0) phi += two_pi;
    const double qf = phi / two_pi * (double)n;
    uint64_t pos = ((uint64_t)floor(qf + 0.5)) & mask;
    if (REF) pos = refine_position(D, L, j, u0r, u0i, rA[j], sigma, n, pos);
    const uint64_t i = (sinv * pos) & mask;
    const BinOffset bo = bin_offset(i, sigma, b, n, B);
    if (bo.h != j) return true;
    const double gp = gprime(-bo.o, n, B, ws);
    if (!(gp >= D.g_min)) return true;
    cv[2 * j] = u0r / gp;
    cv[2 * j + 1] = u0i / gp;
    L.ckey[atomicAdd(&L.misc[1], 1u)] = (i << kCandShift) | j;
    return true;
}

// One round of NoiselessSparseFFTInner on signal `sig` (Algorithm 1).  The
// HBM loads of the round (this lane's first raw bins and zhat values) are
// issued first, so that their latency overlaps the staging.
template <bool REF>
__device__ void exact_round(const DecodeArgs& D, DecodeLds& L, uint32_t sig, uint32_t r, uint64_t seed) {
    const uint32_t tid = threadIdx.x;
    const RoundDev g = D.geom[r];
    const uint64_t n = D.n, mask = n - 1;
    const uint32_t B = g.B;
    const uint64_t sigma = draw_sigma(seed, n, r);
    const uint64_t b = draw_b(seed, n, r);
    const uint64_t sinv = inverse_odd(sigma) & mask;
    const double2* r0 = reinterpret_cast<const double2*>(raw_bins(D, sig, r, 0));
    const double2* r1 = reinterpret_cast<const double2*>(raw_bins(D, sig, r, 1));
    const double2* rA = REF ? reinterpret_cast<const double2*>(raw_bins(D, sig, r, 2)) : nullptr;
    double2 a0[kUnroll], a1[kUnroll];
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; ++u) {
        const uint32_t j = tid + u * kDec;
        if (j < B) {
            a0[u] = r0[j];
            a1[u] = r1[j];
        }
    }
    const uint32_t zc = round_zhat(L, D.zidx, sig, D.capz);
    const double2* zv2 = reinterpret_cast<const double2*>(D.zval + ((uint64_t)sig * 2 + L.sw[ST_ZBUF]) * D.capz * 2);
    double2 zp[kUnroll];
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; ++u) {
        const uint32_t e = tid + u * kDec;
        if (e < zc) zp[u] = zv2[e];
    }
    if (tid == 0) {
        L.misc[0] = 0;
        L.misc[1] = 0;
    }
    double* cv = D.cand_v + (uint64_t)sig * D.Bmax * 2;
    stage_terms(L, zc, zp, zv2, sigma, b, n, B, g.ws);
    uint32_t myJ = 0;
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; ++u) {
        const uint32_t j = tid + u * kDec;
        if (j < B) myJ += exact_bin<REF>(D, L, j, a0[u], a1[u], sigma, sinv, b, n, B, g.ws, cv, rA);
    }
    for (uint32_t j0 = tid + kUnroll * kDec; j0 < B; j0 += kUnroll * kDec) {
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
            const uint32_t j = j0 + u * kDec;
            if (j < B) {
                a0[u] = r0[j];
                a1[u] = r1[j];
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
            const uint32_t j = j0 + u * kDec;
            if (j < B) myJ += exact_bin<REF>(D, L, j, a0[u], a1[u], sigma, sinv, b, n, B, g.ws, cv, rA);
        }
    }
    if (myJ) atomicAdd(&L.misc[0], myJ);
    __syncthreads();
    const uint32_t J = L.misc[0], m = L.misc[1];
    uint32_t* sw = L.sw;
    if (J == 0) {
        // with stop_count, the stop_patience-th empty round in a row ends the
        // signal once that many zhat entries exceed theta/2 (block-uniform:
        // J and the state words are; the barrier below orders these reads
        // before the update of the state words)
        bool enough = false;
        if (D.stop_count && sw[ST_EMPTY] + 1 >= D.stop_patience) {
            const double half = 0.5 * D.theta;
            uint32_t c = 0;
            for (uint32_t e = tid; e < zc; e += kDec) {
                const double2 v = zv2[e];
                c += sqrt(v.x * v.x + v.y * v.y) > half ? 1u : 0u;
            }
            uint32_t pre;
            enough = wave_block_scan(c, L.scan, &pre) >= D.stop_count;
        }
        __syncthreads();
        if (tid == 0) {
            sw[ST_EMPTY] += 1;
            if (sw[ST_EMPTY] >= D.patience || enough) sw[ST_DONE] = 1;
            sw[ST_ROUNDS] = r + 1;
            sw[ST_LASTJ] = 0;
            sw[ST_ACCEPT] = 0;
        }
        __syncthreads();
        return;
    }
    const uint32_t mnew = merge_candidates<true>(L, m, cv, D.zidx, D.zval, sig, D.capz);
    if (tid == 0) {
        sw[ST_EMPTY] = 0;
        sw[ST_ROUNDS] = r + 1;
        sw[ST_LASTJ] = J;
        sw[ST_ACCEPT] = mnew;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kDec) k_exact_init(DecodeArgs D) {
    const uint32_t sig = blockIdx.x * kDec + threadIdx.x;
    if (sig >= D.count) return;
    uint32_t* st = D.state + (uint64_t)sig * kStateWords;
    for (uint32_t q = 0; q < kStateWords; ++q) st[q] = 0;
}

template <bool REF>
__global__ void __launch_bounds__(kDec) k_exact_decode(DecodeArgs D) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t sig = blockIdx.x;
    DecodeLds L = decode_lds(smem, D.capz, D.Bmax, D.gtmp + (uint64_t)sig * D.capz * 4, D.ecount + (uint64_t)sig * D.capz);
    const uint64_t seed = D.seeds ? D.seeds[sig] : D.plan_seed;
    uint32_t* st = D.state + (uint64_t)sig * kStateWords;
    load_state(L, st);
    if (L.sw[ST_DONE]) return;
    stage_zhat(L, D.zidx, sig, D.capz);
    for (uint32_t r = D.r_begin; r < D.r_end; ++r) {
        __syncthreads();
        if (L.sw[ST_DONE]) break;
        exact_round<REF>(D, L, sig, r, seed);
    }
    store_state(L, st);
}

// Final FP64 re-estimation of every zhat entry over the decoded rounds
// (EstimateValues' estimate with a = 0 on x minus the other entries,
// resolved in passes by peel_values), then the output.
__global__ void __launch_bounds__(kDec) k_exact_finish(DecodeArgs D) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t tid = threadIdx.x;
    const uint32_t sig = blockIdx.x;
    DecodeLds L = decode_lds(smem, D.capz, D.Bmax, D.gtmp + (uint64_t)sig * D.capz * 4, D.ecount + (uint64_t)sig * D.capz);
    const uint64_t seed = D.seeds ? D.seeds[sig] : D.plan_seed;
    uint32_t* st = D.state + (uint64_t)sig * kStateWords;
    const uint64_t n = D.n;
    load_state(L, st);
    const uint32_t R = L.sw[ST_ROUNDS];
    const uint32_t zc = stage_zhat(L, D.zidx, sig, D.capz);
    const uint64_t* zi = D.zidx + ((uint64_t)sig * 2 + L.sw[ST_ZBUF]) * D.capz;
    const double* zv = D.zval + ((uint64_t)sig * 2 + L.sw[ST_ZBUF]) * D.capz * 2;
    const double2* zv2 = reinterpret_cast<const double2*>(zv);
    const uint64_t base = (uint64_t)sig * D.rounds * D.capz;
    double* fin = D.fin + (uint64_t)sig * D.capz * 2;
    // zhat of this lane's first entries (fixed), and their raw bins of round 0
    double2 zp[kUnroll], pre[kUnroll];
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; ++u) {
        const uint32_t e = tid + u * kDec;
        if (e < zc) zp[u] = zv2[e];
    }
    if (R > 0) {
        const uint64_t sigma = draw_sigma(seed, n, 0), b = draw_b(seed, n, 0);
        const double2* r0 = reinterpret_cast<const double2*>(raw_bins(D, sig, 0, 0));
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
            const uint32_t e = tid + u * kDec;
            if (e < zc) pre[u] = r0[bin_offset(L.zl[e], sigma, b, n, D.geom[0].B).h];
        }
    }
    for (uint32_t r = 0; r < R; ++r) {
        const RoundDev g = D.geom[r];
        const uint32_t B = g.B;
        const uint64_t sigma = draw_sigma(seed, n, r);
        const uint64_t b = draw_b(seed, n, r);
        __syncthreads();
        // t[2e] = G' zhat_e, t[2e+1].r = G' of entry e
        auto stage = [&](uint32_t e, double2 z) {
            const BinOffset bo = bin_offset(L.zl[e], sigma, b, n, B);
            L.hk[e] = (uint16_t)bo.h;
            const double gp = gprime(-bo.o, n, B, g.ws);
            L.t[2 * e] = cx<double>{gp * z.x, gp * z.y};
            L.t[2 * e + 1] = cx<double>{gp, 0.0};
        };
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u)
            if (tid + u * kDec < zc) stage(tid + u * kDec, zp[u]);
        for (uint32_t e = tid + kUnroll * kDec; e < zc; e += kDec) stage(e, zv2[e]);
        __syncthreads();
        group_by_bin(L, zc, B);
        const double2* r0 = reinterpret_cast<const double2*>(raw_bins(D, sig, r, 0));
        double2 cur[kUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) cur[u] = pre[u];
        if (r + 1 < R) {   // next round's raw bins, in flight during this round's work
            const uint64_t sn = draw_sigma(seed, n, r + 1), bn = draw_b(seed, n, r + 1);
            const uint32_t Bn = D.geom[r + 1].B;
            const double2* rn = reinterpret_cast<const double2*>(raw_bins(D, sig, r + 1, 0));
#pragma unroll
            for (uint32_t u = 0; u < kUnroll; ++u) {
                const uint32_t e = tid + u * kDec;
                if (e < zc) pre[u] = rn[bin_offset(L.zl[e], sn, bn, n, Bn).h];
            }
        }
        const uint64_t row = base + (uint64_t)r * D.capz;
        for (uint32_t q = tid; q < zc; q += kDec) D.eord[row + q] = L.ent[q];
        // the sample table of round r, as k_exact_reest writes it
        auto sample = [&](uint32_t e, double2 a0) {
            const double ge = L.t[2 * e + 1].r;
            const uint32_t h = L.hk[e];
            const uint32_t p0 = L.first[h], p1 = L.first[h + 1];
            if (p1 - p0 > 1) {
                D.egrp[row + e] = p0 << 16 | (p1 - p0);
                D.ecoef[2 * (row + e)] = ge;
                D.ecoef[2 * (row + e) + 1] = 0.0;
            }
            if (ge < D.g_min) {
                D.eflag[row + e] = 0;
                return;
            }
            double orr = 0.0, oii = 0.0;
            for (uint32_t q = p0; q < p1; ++q) {
                const uint32_t e2 = L.ent[q];
                if (e2 == e) continue;
                const cx<double> c2 = L.t[2 * e2];
                orr += c2.r;
                oii += c2.i;
            }
            D.est[2 * (row + e)] = (a0.x - orr) / ge;
            D.est[2 * (row + e) + 1] = (a0.y - oii) / ge;
            D.eflag[row + e] = p1 - p0 == 1 ? 1 : 2;
        };
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u)
            if (tid + u * kDec < zc) sample(tid + u * kDec, cur[u]);
        for (uint32_t e = tid + kUnroll * kDec; e < zc; e += kDec) sample(e, r0[L.hk[e]]);
    }
    __syncthreads();
    const PeelView V{D.est + base * 2, D.eflag + base, D.egrp + base, D.eord + base, D.ecoef + base * 2,
                     D.capz, 1, D.capz, R};
    peel_values<kMaxRounds>(V, zc, zv, fin, L.hk, &L.misc[0], nullptr);
    uint32_t flags = L.sw[ST_FLAGS];
    const uint32_t nout = write_output(L, zi, fin, zc, false, 0.5 * D.theta, D.cap, D.out_scale,
                                       D.out_idx + (uint64_t)sig * D.cap, D.out_val + (uint64_t)sig * D.cap * 2,
                                       &flags);
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

// The same re-estimation split over workgroups, where its LDS fits: round
// r of a signal records its sample table (PeelView: the estimate of every
// zhat entry with the other entries of its bin removed in ascending index
// order, its kind, and for shared bins the grouping and the term
// coefficients); k_exact_output resolves the values and writes the output.
// Each sample is computed exactly as in k_exact_finish.  The tables are
// round-major ([sig][round][capz]) so that both kernels access them
// contiguously across the entries of a wave.
__device__ void reest_round(const DecodeArgs& D, unsigned char* smem, uint32_t sig, uint32_t r) {
    const uint32_t tid = threadIdx.x;
    const uint32_t* st = D.state + (uint64_t)sig * kStateWords;
    const uint32_t zc = st[ST_ZCOUNT], zb = st[ST_ZBUF];
    DecodeLds L;
    reest_lds_layout(D.capz, D.Bmax, smem, &L);
    const uint64_t seed = D.seeds ? D.seeds[sig] : D.plan_seed;
    const uint64_t n = D.n;
    const RoundDev g = D.geom[r];
    const uint32_t B = g.B;
    const uint64_t sigma = draw_sigma(seed, n, r), b = draw_b(seed, n, r);
    const uint64_t* zi = D.zidx + ((uint64_t)sig * 2 + zb) * D.capz;
    const double2* zv2 = reinterpret_cast<const double2*>(D.zval + ((uint64_t)sig * 2 + zb) * D.capz * 2);
    for (uint32_t e = tid; e < zc; e += kDec) {
        const BinOffset bo = bin_offset(zi[e], sigma, b, n, B);
        L.hk[e] = (uint16_t)bo.h;
        const double gp = gprime(-bo.o, n, B, g.ws);
        const double2 z = zv2[e];
        L.t[e] = cx<double>{gp * z.x, gp * z.y};
        L.gp[e] = gp;
    }
    __syncthreads();
    group_by_bin(L, zc, B);
    const double2* r0 = reinterpret_cast<const double2*>(raw_bins(D, sig, r, 0));
    const uint64_t row = ((uint64_t)sig * D.rounds + r) * D.capz;
    double2* est = reinterpret_cast<double2*>(D.est) + row;
    uint8_t* flag = D.eflag + row;
    for (uint32_t q = tid; q < zc; q += kDec) D.eord[row + q] = L.ent[q];
    for (uint32_t e = tid; e < zc; e += kDec) {
        const uint32_t h = L.hk[e];
        const uint32_t p0 = L.first[h], p1 = L.first[h + 1];
        const double ge = L.gp[e];
        if (p1 - p0 > 1) {
            D.egrp[row + e] = p0 << 16 | (p1 - p0);
            D.ecoef[2 * (row + e)] = ge;
            D.ecoef[2 * (row + e) + 1] = 0.0;
        }
        if (ge < D.g_min) {
            flag[e] = 0;
            continue;
        }
        const double2 a0 = r0[h];
        double orr = 0.0, oii = 0.0;
        for (uint32_t q = p0; q < p1; ++q) {
            const uint32_t e2 = L.ent[q];
            if (e2 == e) continue;
            const cx<double> c2 = L.t[e2];
            orr += c2.r;
            oii += c2.i;
        }
        est[e] = make_double2((a0.x - orr) / ge, (a0.y - oii) / ge);
        flag[e] = p1 - p0 == 1 ? 1 : 2;
    }
}

// Blocks per signal of the re-estimation launch: block q takes the rounds
// q, q + 12, ... that the signal decoded.  Most signals stop within 12 or 13
// rounds, so a block mostly does one round; a launch of half the blocks of
// one per (signal, round cap) is dispatched faster next to another stream's
// HashToBins (with four batches in flight, 0.98 against 1.01 ms per batch).
constexpr uint32_t kReestBlocks = 12;

__global__ void __launch_bounds__(kDec) k_exact_reest(DecodeArgs D) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t RB = D.rounds < kReestBlocks ? D.rounds : kReestBlocks;
    const uint32_t sig = blockIdx.x / RB;
    const uint32_t* st = D.state + (uint64_t)sig * kStateWords;
    const uint32_t used = st[ST_ROUNDS];
    for (uint32_t r = blockIdx.x - sig * RB; r < used; r += RB) {
        if (r >= RB) __syncthreads();
        reest_round(D, smem, sig, r);
    }
}

__global__ void __launch_bounds__(kDec) k_exact_output(DecodeArgs D) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t tid = threadIdx.x;
    const uint32_t sig = blockIdx.x;
    DecodeLds L;
    unsigned char* peel_base;
    output_lds_layout(D.capz, D.Bmax, false, smem, &L, &peel_base);
    const PeelScratch P = peel_scratch(peel_base, true);
    uint32_t* st = D.state + (uint64_t)sig * kStateWords;
    load_state(L, st);
    const uint32_t R = L.sw[ST_ROUNDS];
    const uint32_t zc = L.sw[ST_ZCOUNT];
    const uint64_t* zi = D.zidx + ((uint64_t)sig * 2 + L.sw[ST_ZBUF]) * D.capz;
    const double* zv = D.zval + ((uint64_t)sig * 2 + L.sw[ST_ZBUF]) * D.capz * 2;
    const uint64_t base = (uint64_t)sig * D.rounds * D.capz;
    double* fin = D.fin + (uint64_t)sig * D.capz * 2;
    const PeelView V{D.est + base * 2, D.eflag + base, D.egrp + base, D.eord + base, D.ecoef + base * 2,
                     D.capz, 1, D.capz, R};
    peel_values<kMaxRounds>(V, zc, zv, fin, L.hk, &L.misc[0], &P);
    uint32_t flags = L.sw[ST_FLAGS];
    const uint32_t nout = write_output(L, zi, fin, zc, false, 0.5 * D.theta, D.cap, D.out_scale,
                                       D.out_idx + (uint64_t)sig * D.cap, D.out_val + (uint64_t)sig * D.cap * 2,
                                       &flags);
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

// ================================================================= general
__device__ __forceinline__ const double* gen_raw(const GeneralArgs& G, uint32_t sig, uint32_t slot, uint32_t a) {
    return G.raw + (((uint64_t)sig * G.nslots + slot) * 2 + a) * (uint64_t)G.Bmax * 2;
}

// Term spill region of workgroup `part` of signal `sig` (parts: EstimateValues
// hashings or re-estimation rounds), used when LDS cannot hold the terms.
__device__ __forceinline__ double* gen_spill(const GeneralArgs& G, uint32_t sig, uint32_t part) {
    return G.gterm + ((uint64_t)sig * G.nterm + part) * G.capz * 4;
}

// ---- SparseFFT round r (Algorithm 2), split into launches so that the
// independent work of one round (bins of LocateSignal, hashings of
// EstimateValues) spreads over many workgroups:
//   stage (signal) -> locate (signal x bin chunk) -> select (signal)
//   -> estimate (signal x hashing) -> merge (signal)

// LocateSignal staging: for the round's permutation (sigma, b), every zhat
// entry's G'_{-o(i)} zhat_i and sigma i mod n (HBM, [capz][4] doubles) and
// the entries grouped by bin, ascending within a bin; the candidate counter
// reset.
__global__ void __launch_bounds__(kDec) k_gen_stage(GeneralArgs G, uint32_t r) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t tid = threadIdx.x;
    const uint32_t sig = blockIdx.x;
    DecodeLds L = decode_lds(smem, G.capz, G.Bmax, gen_spill(G, sig, 0), G.ecount + (uint64_t)sig * G.capz);
    const uint64_t seed = G.seeds ? G.seeds[sig] : G.plan_seed;
    load_state(L, G.state + (uint64_t)sig * kStateWords);
    const uint64_t n = G.n, mask = n - 1;
    const RoundDev g = G.geom[r];
    const uint32_t B = g.B;
    const uint32_t zc = stage_zhat(L, G.zidx, sig, G.capz);
    const double* zv = G.zval + ((uint64_t)sig * 2 + L.sw[ST_ZBUF]) * G.capz * 2;
    const uint64_t sigma = draw_sigma(seed, n, r, 0, 0);
    const uint64_t b = draw_b(seed, n, r, 0, 0);
    double* zt = G.gtmp + (uint64_t)sig * G.capz * 4;
    uint64_t* zp = reinterpret_cast<uint64_t*>(zt);
    for (uint32_t e = tid; e < zc; e += kDec) {
        const uint64_t i = L.zl[e];
        const BinOffset bo = bin_offset(i, sigma, b, n, B);
        L.hk[e] = (uint16_t)bo.h;
        const double gp = gprime(-bo.o, n, B, g.ws);
        zt[4 * e] = gp * zv[2 * e];
        zt[4 * e + 1] = gp * zv[2 * e + 1];
        zp[4 * e + 2] = (sigma * i) & mask;
    }
    __syncthreads();
    group_by_bin(L, zc, B);
    uint32_t* first = G.gfirst + (uint64_t)sig * (G.Bmax + 1);
    uint32_t* ent = G.gent + (uint64_t)sig * G.capz;
    for (uint32_t h = tid; h <= B; h += kDec) first[h] = L.first[h];
    for (uint32_t q = tid; q < zc; q += kDec) ent[q] = L.ent[q];
    if (tid == 0) G.cand_cnt[sig] = 0;
}

// LocateSignal (Algorithm 3) with LocateInner at every level: one thread per
// bin of round r's hashing, `chunks` workgroups per signal.  Each level
// loads the bin's R_loc measurement pairs first, subtracts the zhat terms of
// the bin (ascending index order), takes the phase of each pair and finds the
// first of the t regions with a majority of votes; a bin that survives every
// level appends its location.
constexpr uint32_t kLoc = 256;

__global__ void __launch_bounds__(kLoc) k_gen_locate(GeneralArgs G, uint32_t r, uint32_t chunks) {
    const uint32_t sig = blockIdx.x / chunks;
    const uint32_t j = (blockIdx.x - sig * chunks) * kLoc + threadIdx.x;
    const RoundDev g = G.geom[r];
    const uint32_t B = g.B;
    if (j >= B) return;
    const GenRoundDev& gr = G.groundv[r];
    const uint64_t seed = G.seeds ? G.seeds[sig] : G.plan_seed;
    const uint64_t n = G.n, mask = n - 1;
    const uint64_t scale = 1ull << kFracBits;
    const uint64_t modfp = n << kFracBits;
    const uint64_t mmask = modfp - 1;
    const double two_pi = 6.283185307179586;
    // 2 pi num / modfp with modfp a power of two: the scaling is exact, so
    // multiplying by 2 pi 2^-m rounds exactly as the division does
    const double ang_scale = ldexp(two_pi, -(int)__builtin_ctzll(modfp));
    const uint64_t sigma = draw_sigma(seed, n, r, 0, 0);
    const uint64_t b = draw_b(seed, n, r, 0, 0);
    const uint64_t sinv = inverse_odd(sigma) & mask;
    const uint64_t sbs = ((sigma * b) & mask) << kFracBits;
    const double tol = G.s * 3.141592653589793;
    const double* zt = G.gtmp + (uint64_t)sig * G.capz * 4;
    const uint64_t* zp = reinterpret_cast<const uint64_t*>(zt);
    const uint32_t* ent = G.gent + (uint64_t)sig * G.capz;
    const uint32_t q0 = G.gfirst[(uint64_t)sig * (G.Bmax + 1) + j];
    const uint32_t q1 = G.gfirst[(uint64_t)sig * (G.Bmax + 1) + j + 1];
    const uint32_t R_loc = G.R_loc, t = G.t;
    uint64_t l = ((uint64_t)j * (n / B) * scale + modfp - (n / (2 * (uint64_t)B)) * scale) & mmask;
    for (uint32_t D = 1; D <= gr.nlev; ++D) {
        const uint64_t W = gr.Wfp[D - 1];
        const uint64_t half = W / (2 * (uint64_t)t);
        const uint64_t step = W / t;
        double2 u0[kMaxRLoc], u1[kMaxRLoc];
#pragma unroll
        for (uint32_t q = 0; q < kMaxRLoc; ++q)
            if (q < R_loc) {
                const uint32_t slot = gr.slot0 + (D - 1) * R_loc + q;
                u0[q] = reinterpret_cast<const double2*>(gen_raw(G, sig, slot, 0))[j];
                u1[q] = reinterpret_cast<const double2*>(gen_raw(G, sig, slot, 1))[j];
            }
        double ph[kMaxRLoc];
        uint64_t bet[kMaxRLoc];
#pragma unroll
        for (uint32_t q = 0; q < kMaxRLoc; ++q)
            if (q < R_loc) {
                const uint64_t a = draw_a(seed, n, r, D, q);
                const uint64_t beta = draw_beta(seed, gr.blo[D - 1], gr.bhi[D - 1], r, D, q);
                const uint64_t ab = (a + beta) & mask;
                cx<double> u{u0[q].x, u0[q].y}, u2{u1[q].x, u1[q].y};
                for (uint32_t qq = q0; qq < q1; ++qq) {
                    const uint32_t e = ent[qq];
                    const cx<double> c0{zt[4 * e], zt[4 * e + 1]};
                    const uint64_t p = zp[4 * e + 2];
                    u = csub(u, cmul(c0, omega_d((a * p) & mask, n)));
                    u2 = csub(u2, cmul(c0, omega_d((ab * p) & mask, n)));
                }
                ph[q] = phase_of(u, u2);
                bet[q] = beta;
            }
        uint32_t firstq = t;
        for (uint32_t qq = 0; qq < t; ++qq) {
            const uint64_t M = (l + (2 * (uint64_t)qq + 1) * half) & mmask;
            uint32_t votes = 0;
#pragma unroll
            for (uint32_t q = 0; q < kMaxRLoc; ++q)
                if (q < R_loc) {
                    const uint64_t num = (bet[q] * ((M + sbs) & mmask)) & mmask;
                    const double ang = (double)num * ang_scale;
                    const double d = fabs(ang - ph[q]);
                    const double dist = d < two_pi - d ? d : two_pi - d;
                    votes += dist < tol;
                }
            if (2u * votes > R_loc) {
                firstq = qq;
                break;
            }
        }
        if (firstq == t) return;
        l = (l + firstq * step) & mmask;
    }
    const uint64_t pos = ((l + scale - 1) >> kFracBits) & mask;
    const uint32_t at = atomicAdd(&G.cand_cnt[sig], 1u);
    G.cand_raw[(uint64_t)sig * G.Bmax + at] = (sinv * pos + b) & mask;
}

// The located candidates of a signal sorted, duplicates removed (G.cand_i,
// count in G.cand_cnt); measurement masks cleared.
__global__ void __launch_bounds__(kDec) k_gen_select(GeneralArgs G) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t tid = threadIdx.x;
    const uint32_t sig = blockIdx.x;
    DecodeLds L = decode_lds(smem, G.capz, G.Bmax, gen_spill(G, sig, 0), G.ecount + (uint64_t)sig * G.capz);
    uint64_t* cand = G.cand_i + (uint64_t)sig * G.Bmax;
    const uint32_t m = G.cand_cnt[sig];
    const uint32_t NM = pow2_ceil_u32(m > 0 ? m : 1);
    const uint64_t* raw = G.cand_raw + (uint64_t)sig * G.Bmax;
    for (uint32_t q = tid; q < NM; q += kDec) L.ckey[q] = q < m ? raw[q] : kNone;
    bitonic_sort_u64<kDec>(L.ckey, NM);
    const uint32_t per = (m + kDec - 1) / kDec;
    const uint32_t p0 = tid * per < m ? tid * per : m;
    const uint32_t p1 = p0 + per < m ? p0 + per : m;
    uint32_t cnt = 0;
    for (uint32_t p = p0; p < p1; ++p) cnt += (p == 0 || L.ckey[p] != L.ckey[p - 1]);
    uint32_t pre;
    const uint32_t nL = wave_block_scan(cnt, L.scan, &pre);
    for (uint32_t p = p0; p < p1; ++p)
        if (p == 0 || L.ckey[p] != L.ckey[p - 1]) cand[pre++] = L.ckey[p];
    uint32_t* mk = G.cand_n + (uint64_t)sig * G.Bmax;
    for (uint32_t c = tid; c < nL; c += kDec) mk[c] = 0;
    __syncthreads();
    if (tid == 0) G.cand_cnt[sig] = nL;
}

// EstimateValues (Algorithm 2), hashing e of round r for every candidate of
// one signal (one workgroup per signal and hashing): the estimate
// (u_h - zhat terms of bin h) omega^{-a sigma i} / G'_{-o(i)} where
// G' >= g_min, recorded in slot e with bit e of the candidate's mask.
__global__ void __launch_bounds__(kDec) k_gen_estimate(GeneralArgs G, uint32_t r) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t tid = threadIdx.x;
    const uint32_t sig = blockIdx.x / G.R_est;
    const uint32_t e = blockIdx.x - sig * G.R_est;
    DecodeLds L = decode_lds(smem, G.capz, G.Bmax, gen_spill(G, sig, e), G.ecount + (uint64_t)sig * G.capz);
    const uint64_t seed = G.seeds ? G.seeds[sig] : G.plan_seed;
    load_state(L, G.state + (uint64_t)sig * kStateWords);
    const uint64_t n = G.n, mask = n - 1;
    const RoundDev g = G.geom[r];
    const GenRoundDev& gr = G.groundv[r];
    const uint32_t B = g.B;
    const uint32_t zc = stage_zhat(L, G.zidx, sig, G.capz);
    const double* zv = G.zval + ((uint64_t)sig * 2 + L.sw[ST_ZBUF]) * G.capz * 2;
    const uint64_t sigma = draw_sigma(seed, n, r, LEVEL_EST, e);
    const uint64_t a = draw_a(seed, n, r, LEVEL_EST, e);
    const uint64_t b = draw_b(seed, n, r, LEVEL_EST, e);
    const uint64_t as = (a * sigma) & mask;
    const double* rawv = gen_raw(G, sig, gr.slot0 + gr.nloc + e, 0);
    for (uint32_t q = tid; q < zc; q += kDec) {
        const uint64_t i = L.zl[q];
        const BinOffset bo = bin_offset(i, sigma, b, n, B);
        L.hk[q] = (uint16_t)bo.h;
        const double gp = gprime(-bo.o, n, B, g.ws);
        const cx<double> c0{gp * zv[2 * q], gp * zv[2 * q + 1]};
        L.t[2 * q] = cmul(c0, omega_d((as * i) & mask, n));
    }
    __syncthreads();
    group_by_bin(L, zc, B);
    const uint32_t nL = G.cand_cnt[sig];
    const uint64_t* cand = G.cand_i + (uint64_t)sig * G.Bmax;
    uint32_t* mk = G.cand_n + (uint64_t)sig * G.Bmax;
    for (uint32_t c = tid; c < nL; c += kDec) {
        const uint64_t i = cand[c];
        const BinOffset bo = bin_offset(i, sigma, b, n, B);
        const double gp = gprime(-bo.o, n, B, g.ws);
        if (gp < G.g_min) continue;
        const uint32_t h = bo.h;
        cx<double> u{rawv[2 * h], rawv[2 * h + 1]};
        for (uint32_t q = L.first[h]; q < L.first[h + 1]; ++q) u = csub(u, L.t[2 * L.ent[q]]);
        const uint64_t p = (as * i) & mask;
        const cx<double> v = cmul(u, omega_d((n - p) & mask, n));
        double* dst = G.cand_e + (((uint64_t)sig * G.Bmax + c) * G.R_est + e) * 2;
        dst[0] = v.r / gp;
        dst[1] = v.i / gp;
        atomicOr(&mk[c], 1u << e);
    }
}

// Medians of each candidate's estimates, the top 3 k_r by (|w| desc, index
// asc), and their merge into zhat (one workgroup per signal).
__global__ void __launch_bounds__(kDec) k_gen_merge(GeneralArgs G, uint32_t r) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t tid = threadIdx.x;
    const uint32_t sig = blockIdx.x;
    DecodeLds L = decode_lds(smem, G.capz, G.Bmax, gen_spill(G, sig, 0), G.ecount + (uint64_t)sig * G.capz);
    uint32_t* st = G.state + (uint64_t)sig * kStateWords;
    load_state(L, st);
    const GenRoundDev& gr = G.groundv[r];
    stage_zhat(L, G.zidx, sig, G.capz);
    const uint32_t nL = G.cand_cnt[sig];
    const uint64_t* cand = G.cand_i + (uint64_t)sig * G.Bmax;
    double* candv = G.cand_v + (uint64_t)sig * G.Bmax * 2;
    uint32_t* mk = G.cand_n + (uint64_t)sig * G.Bmax;
    for (uint32_t c = tid; c < nL; c += kDec) {
        // the valid estimates to the front, in hashing order
        double* src = G.cand_e + ((uint64_t)sig * G.Bmax + c) * G.R_est * 2;
        const uint32_t bits = mk[c];
        uint32_t k = 0;
        for (uint32_t e = 0; e < G.R_est; ++e)
            if (bits & (1u << e)) {
                if (k != e) {
                    src[2 * k] = src[2 * e];
                    src[2 * k + 1] = src[2 * e + 1];
                }
                ++k;
            }
        mk[c] = k;
        if (k == 0) continue;
        const cx<double> med = median_cx<kMaxREst>(src, k);
        candv[2 * c] = med.r;
        candv[2 * c + 1] = med.i;
    }
    __syncthreads();
    const uint32_t kprime = 3 * gr.k_r;
    const uint32_t NL = pow2_ceil_u32(nL > 0 ? nL : 1);
    for (uint32_t c = tid; c < NL; c += kDec)
        L.ckey[c] = (c < nL && mk[c] > 0) ? mag_key(candv[2 * c], candv[2 * c + 1], c) : kNone;
    bitonic_sort_u64<kDec>(L.ckey, NL);
    uint32_t take = 0;
    {
        uint32_t mine = 0;
        for (uint32_t q = tid; q < NL; q += kDec) mine += (q < kprime && L.ckey[q] != kNone);
        if (tid == 0) L.misc[1] = 0;
        __syncthreads();
        if (mine) atomicAdd(&L.misc[1], mine);
        __syncthreads();
        take = L.misc[1];
    }
    for (uint32_t q = tid; q < take; q += kDec) {
        const uint32_t c = (uint32_t)(L.ckey[q] & kSlotMask);
        L.ckey[q] = (cand[c] << kCandShift) | c;
    }
    __syncthreads();
    merge_candidates<false>(L, take, candv, G.zidx, G.zval, sig, G.capz);
    if (tid == 0) {
        L.sw[ST_ROUNDS] = r + 1;
        L.sw[ST_LASTJ] = nL;
    }
    store_state(L, st);
}

// Final FP64 re-estimation, round r (one workgroup per signal and round): for
// each EstimateValues hashing of the round, every zhat entry's estimate with
// the other entries of its bin removed, flagged isolated (alone in its bin) or
// crowded.
__global__ void __launch_bounds__(kDec) k_gen_reest(GeneralArgs G) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t tid = threadIdx.x;
    const uint32_t sig = blockIdx.x / G.R;
    const uint32_t r = blockIdx.x - sig * G.R;
    DecodeLds L = decode_lds(smem, G.capz, G.Bmax, gen_spill(G, sig, r), G.ecount + (uint64_t)sig * G.capz);
    const uint64_t seed = G.seeds ? G.seeds[sig] : G.plan_seed;
    load_state(L, G.state + (uint64_t)sig * kStateWords);
    if (r >= L.sw[ST_ROUNDS]) return;
    const uint64_t n = G.n, mask = n - 1;
    const RoundDev g = G.geom[r];
    const GenRoundDev& gr = G.groundv[r];
    const uint32_t B = g.B;
    const uint32_t zc = stage_zhat(L, G.zidx, sig, G.capz);
    const double* zv = G.zval + ((uint64_t)sig * 2 + L.sw[ST_ZBUF]) * G.capz * 2;
    const uint32_t nmeas = G.R * G.R_est;
    double* est = G.est + (uint64_t)sig * G.capz * nmeas * 2;
    uint8_t* flag = G.eflag + (uint64_t)sig * G.capz * nmeas;
    for (uint32_t m = 0; m < G.R_est; ++m) {
        const uint64_t sigma = draw_sigma(seed, n, r, LEVEL_EST, m);
        const uint64_t a = draw_a(seed, n, r, LEVEL_EST, m);
        const uint64_t b = draw_b(seed, n, r, LEVEL_EST, m);
        const double* rawv = gen_raw(G, sig, gr.slot0 + gr.nloc + m, 0);
        const uint64_t as = (a * sigma) & mask;
        const uint32_t meas = r * G.R_est + m;
        __syncthreads();
        // t[2e] = G' zhat_e omega^{a sigma i_e}, t[2e+1].r = G' of entry e
        for (uint32_t e = tid; e < zc; e += kDec) {
            const BinOffset bo = bin_offset(L.zl[e], sigma, b, n, B);
            L.hk[e] = (uint16_t)bo.h;
            const double gp = gprime(-bo.o, n, B, g.ws);
            const cx<double> c0{gp * zv[2 * e], gp * zv[2 * e + 1]};
            L.t[2 * e] = cmul(c0, omega_d((as * L.zl[e]) & mask, n));
            L.t[2 * e + 1] = cx<double>{gp, 0.0};
        }
        __syncthreads();
        group_by_bin(L, zc, B);
        uint16_t* ord = G.eord + ((uint64_t)sig * nmeas + meas) * G.capz;
        for (uint32_t q = tid; q < zc; q += kDec) ord[q] = L.ent[q];
        const uint64_t base = (uint64_t)sig * G.capz * nmeas + meas;
        for (uint32_t e = tid; e < zc; e += kDec) {
            const double ge = L.t[2 * e + 1].r;
            const uint32_t h = L.hk[e];
            const uint32_t p0 = L.first[h], p1 = L.first[h + 1];
            const uint64_t slot = base + (uint64_t)e * nmeas;
            const uint64_t pe = (as * L.zl[e]) & mask;
            if (p1 - p0 > 1) {
                const cx<double> c = cmul(cx<double>{ge, 0.0}, omega_d(pe, n));
                G.egrp[slot] = p0 << 16 | (p1 - p0);
                G.ecoef[2 * slot] = c.r;
                G.ecoef[2 * slot + 1] = c.i;
            }
            if (ge < G.g_min) {
                flag[(uint64_t)e * nmeas + meas] = 0;
                continue;
            }
            cx<double> others{0.0, 0.0};
            for (uint32_t q = p0; q < p1; ++q) {
                const uint32_t e2 = L.ent[q];
                if (e2 == e) continue;
                others = cadd(others, L.t[2 * e2]);
            }
            const cx<double> u = csub(cx<double>{rawv[2 * h], rawv[2 * h + 1]}, others);
            const cx<double> v = cmul(u, omega_d((n - pe) & mask, n));
            double* dst = est + ((uint64_t)e * nmeas + meas) * 2;
            dst[0] = v.r / ge;
            dst[1] = v.i / ge;
            flag[(uint64_t)e * nmeas + meas] = p1 - p0 == 1 ? 1 : 2;
        }
    }
}

// Medians over every entry's re-estimation samples (isolated ones when there
// are any, else the crowded ones), then the top-cap entries by magnitude in
// ascending index order (one workgroup per signal).
__global__ void __launch_bounds__(kDec) k_gen_output(GeneralArgs G) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t tid = threadIdx.x;
    const uint32_t sig = blockIdx.x;
    DecodeLds L;
    unsigned char* peel_base;
    output_lds_layout(G.capz, G.Bmax, true, smem, &L, &peel_base);
    const PeelScratch P = peel_scratch(peel_base, false);
    uint32_t* st = G.state + (uint64_t)sig * kStateWords;
    load_state(L, st);
    const uint32_t R = L.sw[ST_ROUNDS];
    const uint32_t zc = stage_zhat(L, G.zidx, sig, G.capz);
    const uint64_t* zi = G.zidx + ((uint64_t)sig * 2 + L.sw[ST_ZBUF]) * G.capz;
    const double* zv = G.zval + ((uint64_t)sig * 2 + L.sw[ST_ZBUF]) * G.capz * 2;
    const uint32_t nmeas = G.R * G.R_est;
    const uint32_t used = (R < G.R ? R : G.R) * G.R_est;
    const uint64_t base = (uint64_t)sig * G.capz * nmeas;
    double* fin = G.fin + (uint64_t)sig * G.capz * 2;
    const PeelView V{G.est + base * 2, G.eflag + base, G.egrp + base, G.eord + base, G.ecoef + base * 2,
                     1, nmeas, G.capz, used};
    peel_values<kMaxMeas>(V, zc, zv, fin, L.hk, &L.misc[0], &P);
    uint32_t flags = L.sw[ST_FLAGS];
    const uint32_t nout = write_output(L, zi, fin, zc, true, 0.0, G.cap, G.out_scale,
                                       G.out_idx + (uint64_t)sig * G.cap, G.out_val + (uint64_t)sig * G.cap * 2,
                                       &flags);
    if (tid == 0) {
        G.out_count[sig] = nout;
        if (G.out_info) {
            G.out_info[(uint64_t)sig * 4 + SFFT_INFO_ROUNDS] = R;
            G.out_info[(uint64_t)sig * 4 + SFFT_INFO_FLAGS] = flags;
            G.out_info[(uint64_t)sig * 4 + SFFT_INFO_ZHAT] = zc;
            G.out_info[(uint64_t)sig * 4 + SFFT_INFO_LOCATED] = L.sw[ST_LASTJ];
        }
    }
}

// ------------------------------------------------------------------ launch --
hipError_t launch_exact_init(const DecodeArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_exact_init, dim3((a.count + kDec - 1) / kDec), dim3(kDec), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_exact_decode(const DecodeArgs& a, hipStream_t s) {
    const size_t lds = decode_lds_bytes(a.capz, a.Bmax);
    if (a.refine_shift) {
        hipError_t e = allow_lds(k_exact_decode<true>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_exact_decode<true>, dim3(a.count), dim3(kDec), lds, s, a);
        return hipGetLastError();
    }
    hipError_t e = allow_lds(k_exact_decode<false>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_exact_decode<false>, dim3(a.count), dim3(kDec), lds, s, a);
    return hipGetLastError();
}

// The split re-estimation (signal x round workgroups, then one output
// workgroup per signal) where its LDS fits, else one workgroup per signal.
hipError_t launch_exact_finish(const DecodeArgs& a, hipStream_t s) {
    const size_t lds = decode_lds_bytes(a.capz, a.Bmax);
    const size_t rlds = reest_lds_bytes(a.capz, a.Bmax);
    const size_t olds = output_lds_bytes(a.capz, a.Bmax, false);
    if (rlds <= kLdsLimit && olds <= kLdsLimit) {
        hipError_t e = allow_lds(k_exact_reest, rlds);
        if (e != hipSuccess) return e;
        e = allow_lds(k_exact_output, olds);
        if (e != hipSuccess) return e;
        const uint32_t rb = a.rounds < kReestBlocks ? a.rounds : kReestBlocks;
        hipLaunchKernelGGL(k_exact_reest, dim3(a.count * rb), dim3(kDec), rlds, s, a);
        hipLaunchKernelGGL(k_exact_output, dim3(a.count), dim3(kDec), olds, s, a);
        return hipGetLastError();
    }
    hipError_t e = allow_lds(k_exact_finish, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_exact_finish, dim3(a.count), dim3(kDec), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_general_decode(const GeneralArgs& a, uint32_t r_begin, uint32_t r_end, hipStream_t s) {
    const size_t lds = decode_lds_bytes(a.capz, a.Bmax);
    for (auto k : {k_gen_stage, k_gen_merge}) {
        hipError_t e = allow_lds(k, lds);
        if (e != hipSuccess) return e;
    }
    for (auto k : {k_gen_select, k_gen_reest}) {
        hipError_t e = allow_lds(k, lds);
        if (e != hipSuccess) return e;
    }
    hipError_t e = allow_lds(k_gen_estimate, lds);
    if (e != hipSuccess) return e;
    const uint32_t chunks = (a.Bmax + kLoc - 1) / kLoc;
    for (uint32_t r = r_begin; r < r_end; ++r) {
        hipLaunchKernelGGL(k_gen_stage, dim3(a.count), dim3(kDec), lds, s, a, r);
        hipLaunchKernelGGL(k_gen_locate, dim3(a.count * chunks), dim3(kLoc), 0, s, a, r, chunks);
        hipLaunchKernelGGL(k_gen_select, dim3(a.count), dim3(kDec), lds, s, a);
        hipLaunchKernelGGL(k_gen_estimate, dim3(a.count * a.R_est), dim3(kDec), lds, s, a, r);
        hipLaunchKernelGGL(k_gen_merge, dim3(a.count), dim3(kDec), lds, s, a, r);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_general_finish(const GeneralArgs& a, hipStream_t s) {
    const size_t lds = decode_lds_bytes(a.capz, a.Bmax);
    const size_t olds = output_lds_bytes(a.capz, a.Bmax, true);
    hipError_t e = allow_lds(k_gen_reest, lds);
    if (e != hipSuccess) return e;
    e = allow_lds(k_gen_output, olds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gen_reest, dim3(a.count * a.R), dim3(kDec), lds, s, a);
    hipLaunchKernelGGL(k_gen_output, dim3(a.count), dim3(kDec), olds, s, a);
    return hipGetLastError();
}

}  // namespace sfft
