// Dense fallback of the serving runtime: after a full-length FFT of each
// signal, keep the `cap` bins of largest magnitude (ties: the smaller index),
// in ascending index order.  Used where the sparse plan would gather about as
// much as the whole signal, so the sparse method has nothing to save.
//
// Radix select on the FP32 bit pattern of |X_f|^2 (non-negative floats order
// as unsigned integers), spread over the chip: each spectrum is cut into nb
// contiguous chunks, one 256-thread workgroup per chunk.  Four 8-bit passes
// (each a histogram of the keys that match the prefix found so far; the
// next pass's workgroups, and after the last one the counting workgroups,
// first walk that histogram to extend the prefix) find the key T of the
// cap-th largest bin and how many bins equal to T are taken (the smallest
// indices).  Then every chunk counts the bins it keeps, one workgroup per
// spectrum scans the counts into output offsets, and every chunk writes its
// kept bins in index order.  Kept: key > T, and the first take_eq bins with key == T;
// with keep_above >= 0 only bins whose key exceeds that of keep_above.
#include <cstring>
#include <mutex>

#include "sfft_device.hpp"

namespace sfft {

namespace {

constexpr uint32_t kTk = 256;              // threads per workgroup
constexpr uint32_t kTkMaxChunks = 1024;    // chunks per spectrum at most
constexpr uint32_t kTkMinChunk = 4096;     // bins per chunk at least (when n allows)
// scratch words per spectrum: the four passes' histograms; the selection
// state after 0..4 digits (prefix, mask, need; one slot each, so that no
// workgroup reads a slot another one is writing); the whole-spectrum flag;
// per-chunk counts and offsets
constexpr uint32_t kTkHist = 0, kTkState = 4 * 256, kTkAll = kTkState + 5 * 4, kTkCnt = kTkAll + 4;
constexpr uint32_t kTkOff = kTkCnt + 2 * kTkMaxChunks;
constexpr uint32_t kTkStride = kTkOff + 2 * kTkMaxChunks;
constexpr uint32_t ST_PREFIX = 0, ST_MASK = 1, ST_NEED = 2;

// The key of a bin, with the rounding spelled out so that every kernel
// computes the same bits.
__device__ __forceinline__ uint32_t mag_bits(float2 v) {
    return __float_as_uint(__fmaf_rn(v.x, v.x, __fmul_rn(v.y, v.y)));
}

// Exclusive prefix of one value per thread over the 256-thread block;
// returns the block total.  wsum: 4 words of LDS.
__device__ uint32_t block_scan_256(uint32_t v, uint32_t* wsum, uint32_t* prefix) {
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    uint32_t inc = v;
#pragma unroll
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    __syncthreads();
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (uint32_t w = 0; w < kTk / 64; ++w) {
        const uint32_t c = wsum[w];
        before += w < wave ? c : 0u;
        total += c;
    }
    *prefix = before + inc - v;
    return total;
}

__device__ __forceinline__ uint32_t block_sum_256(uint32_t v, uint32_t* wsum) {
    uint32_t pre;
    return block_scan_256(v, wsum, &pre);
}

__global__ void __launch_bounds__(kTk) k_topk_init(uint32_t* scratch, uint64_t n, uint32_t cap) {
    uint32_t* sc = scratch + (size_t)blockIdx.x * kTkStride;
    for (uint32_t d = threadIdx.x; d < 4 * 256; d += kTk) sc[kTkHist + d] = 0;
    if (threadIdx.x == 0) {
        sc[kTkState + ST_PREFIX] = 0;
        sc[kTkState + ST_MASK] = 0;
        sc[kTkState + ST_NEED] = cap;
        sc[kTkAll] = (uint64_t)cap >= n ? 1u : 0u;
    }
}

// The selection state after digit p: the state before it (slot p) extended
// by the bucket of pass p's histogram that holds the need-th largest
// matching key.  The histogram is staged in LDS and walked by thread 0;
// every thread gets the result in st[0..2].
__device__ void tk_extend(const uint32_t* sc, uint32_t p, uint32_t* walk, uint32_t* st) {
    walk[threadIdx.x] = sc[kTkHist + 256 * p + threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t* before = sc + kTkState + 4 * p;
        const uint32_t need = before[ST_NEED];
        uint32_t acc = 0, digit = 0;
        for (int d = 255; d >= 0; --d) {
            const uint32_t h = walk[d];
            if (acc + h >= need) {
                digit = (uint32_t)d;
                break;
            }
            acc += h;
        }
        const uint32_t shift = 24 - 8 * p;
        st[ST_PREFIX] = before[ST_PREFIX] | (digit << shift);
        st[ST_MASK] = before[ST_MASK] | (255u << shift);
        st[ST_NEED] = need - acc;
    }
    __syncthreads();
}

// Pass p: histogram of digit p over the keys of this chunk that match the
// prefix of digits 0..p-1 (extended here from pass p-1's histogram; chunk 0
// stores it in slot p); one LDS histogram per wave, summed into the
// spectrum's histogram of pass p.
__global__ void __launch_bounds__(kTk) k_topk_hist(const float2* __restrict__ spec, uint64_t n, uint64_t chunk,
                                                   uint32_t* scratch, uint32_t p) {
    __shared__ uint32_t hist[kTk / 64][256];
    __shared__ uint32_t walk[256];
    __shared__ uint32_t st[3];
    const uint32_t tid = threadIdx.x, wave = tid >> 6;
    const uint32_t sig = blockIdx.y;
    uint32_t* sc = scratch + (size_t)sig * kTkStride;
    if (sc[kTkAll]) return;
    uint32_t prefix = 0, mask = 0;
    if (p > 0) {
        tk_extend(sc, p - 1, walk, st);
        prefix = st[ST_PREFIX];
        mask = st[ST_MASK];
        if (blockIdx.x == 0 && tid < 3) sc[kTkState + 4 * p + tid] = st[tid];
    }
    const uint32_t shift = 24 - 8 * p;
    for (uint32_t d = tid; d < 256 * (kTk / 64); d += kTk) (&hist[0][0])[d] = 0;
    __syncthreads();
    const float2* x = spec + (size_t)sig * n + (size_t)blockIdx.x * chunk;
    for (uint64_t f = tid; f < chunk; f += kTk) {
        const uint32_t k = mag_bits(x[f]);
        if ((k & mask) == prefix) atomicAdd(&hist[wave][(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    uint32_t c = 0;
#pragma unroll
    for (uint32_t w = 0; w < kTk / 64; ++w) c += hist[w][tid];
    if (c) atomicAdd(&sc[kTkHist + 256 * p + tid], c);
}

struct TkSel {
    uint32_t T, take_eq;
};

// The final selection (slot 4, stored by the counting kernel).
__device__ __forceinline__ TkSel tk_selection(const uint32_t* sc) {
    if (sc[kTkAll]) return {0u, 0xFFFFFFFFu};
    return {sc[kTkState + 16 + ST_PREFIX], sc[kTkState + 16 + ST_NEED]};
}

// Per chunk: bins above T that are kept, and bins equal to T (T and the
// ties to take from the last pass's histogram; chunk 0 stores them).
__global__ void __launch_bounds__(kTk) k_topk_count(const float2* __restrict__ spec, uint64_t n, uint64_t chunk,
                                                    uint32_t* scratch, uint32_t keep_all, uint32_t KT) {
    __shared__ uint32_t wsum[kTk / 64];
    __shared__ uint32_t walk[256];
    __shared__ uint32_t st[3];
    const uint32_t sig = blockIdx.y;
    uint32_t* sc = scratch + (size_t)sig * kTkStride;
    TkSel s = {0u, 0xFFFFFFFFu};
    if (!sc[kTkAll]) {
        tk_extend(sc, 3, walk, st);
        s = {st[ST_PREFIX], st[ST_NEED]};
        if (blockIdx.x == 0 && threadIdx.x < 3) sc[kTkState + 16 + threadIdx.x] = st[threadIdx.x];
    }
    const float2* x = spec + (size_t)sig * n + (size_t)blockIdx.x * chunk;
    uint32_t gt = 0, eq = 0;
    for (uint64_t f = threadIdx.x; f < chunk; f += kTk) {
        const uint32_t k = mag_bits(x[f]);
        gt += (k > s.T && (keep_all || k > KT)) ? 1u : 0u;
        eq += k == s.T ? 1u : 0u;
    }
    gt = block_sum_256(gt, wsum);
    eq = block_sum_256(eq, wsum);
    if (threadIdx.x == 0) {
        sc[kTkCnt + 2 * blockIdx.x] = gt;
        sc[kTkCnt + 2 * blockIdx.x + 1] = eq;
    }
}

// One workgroup per spectrum: output offset and bins equal to T before each
// chunk, the spectrum's count, and zeros in the unused output slots.
__global__ void __launch_bounds__(kTk) k_topk_scan(uint32_t* scratch, uint32_t nb, uint32_t cap, uint32_t keep_all,
                                                   uint32_t KT, uint64_t* out_idx, double* out_val,
                                                   uint32_t* out_count) {
    __shared__ uint32_t wsum[kTk / 64];
    const uint32_t sig = blockIdx.x, tid = threadIdx.x;
    uint32_t* sc = scratch + (size_t)sig * kTkStride;
    const TkSel s = tk_selection(sc);
    const bool eq_keep = keep_all || s.T > KT;
    uint32_t eq_run = 0, out_run = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += kTk) {
        const uint32_t b = b0 + tid;
        const uint32_t gt = b < nb ? sc[kTkCnt + 2 * b] : 0u;
        const uint32_t eq = b < nb ? sc[kTkCnt + 2 * b + 1] : 0u;
        uint32_t eq_pre;
        const uint32_t eq_tot = block_scan_256(eq, wsum, &eq_pre);
        const uint32_t eq_before = eq_run + eq_pre;
        const uint32_t left = s.take_eq > eq_before ? s.take_eq - eq_before : 0u;
        const uint32_t taken = eq_keep ? min(left, eq) : 0u;
        uint32_t out_pre;
        const uint32_t out_tot = block_scan_256(gt + taken, wsum, &out_pre);
        if (b < nb) {
            sc[kTkOff + 2 * b] = out_run + out_pre;
            sc[kTkOff + 2 * b + 1] = eq_before;
        }
        eq_run += eq_tot;
        out_run += out_tot;
    }
    const uint32_t total = min(out_run, cap);
    uint64_t* oi = out_idx + (size_t)sig * cap;
    double* ov = out_val + (size_t)sig * cap * 2;
    for (uint32_t q = total + tid; q < cap; q += kTk) {
        oi[q] = 0;
        ov[2 * q] = 0.0;
        ov[2 * q + 1] = 0.0;
    }
    if (tid == 0) out_count[sig] = total;
}

// Per chunk, in index order: the kept bins at their output offsets.
__global__ void __launch_bounds__(kTk) k_topk_write(const float2* __restrict__ spec, uint64_t n, uint64_t chunk,
                                                    const uint32_t* __restrict__ scratch, uint32_t cap,
                                                    uint32_t keep_all, uint32_t KT, double scale,
                                                    uint64_t* out_idx, double* out_val) {
    __shared__ uint32_t wsum[kTk / 64];
    const uint32_t sig = blockIdx.y, b = blockIdx.x, tid = threadIdx.x;
    const uint32_t* sc = scratch + (size_t)sig * kTkStride;
    const TkSel s = tk_selection(sc);
    const bool eq_keep = keep_all || s.T > KT;
    const uint32_t off = sc[kTkOff + 2 * b], eq_before = sc[kTkOff + 2 * b + 1];
    // a chunk that keeps nothing writes nothing
    const uint32_t gt_here = sc[kTkCnt + 2 * b], eq_here = sc[kTkCnt + 2 * b + 1];
    if (gt_here == 0 && (!eq_keep || eq_here == 0 || eq_before >= s.take_eq)) return;
    const uint64_t base0 = (uint64_t)b * chunk;
    const float2* x = spec + (size_t)sig * n + base0;
    uint64_t* oi = out_idx + (size_t)sig * cap;
    double* ov = out_val + (size_t)sig * cap * 2;
    uint32_t written = 0, ties = 0;
    for (uint64_t t0 = 0; t0 < chunk; t0 += kTk) {
        const float2 v = x[t0 + tid];
        const uint32_t k = mag_bits(v);
        const bool gt = k > s.T && (keep_all || k > KT);
        const bool eq = k == s.T;
        // a tile with no bin at or above T moves no counter: skip its scans
        if (!__syncthreads_or((gt || eq) ? 1 : 0)) continue;
        uint32_t tie_pre;
        const uint32_t tie_tot = block_scan_256(eq ? 1u : 0u, wsum, &tie_pre);
        const bool keep = gt || (eq && eq_keep && eq_before + ties + tie_pre < s.take_eq);
        uint32_t pos;
        const uint32_t kept = block_scan_256(keep ? 1u : 0u, wsum, &pos);
        const uint32_t q = off + written + pos;
        if (keep && q < cap) {
            oi[q] = base0 + t0 + tid;
            ov[2 * q] = (double)v.x * scale;
            ov[2 * q + 1] = (double)v.y * scale;
        }
        written += kept;
        ties += tie_tot;
    }
}

uint32_t topk_chunks(uint64_t n) {
    uint64_t nb = n / kTkMinChunk;
    nb = nb < 1 ? 1 : (nb > kTkMaxChunks ? kTkMaxChunks : nb);
    return (uint32_t)nb;
}

}  // namespace

size_t dense_topk_scratch_bytes(uint32_t count) { return (size_t)count * kTkStride * sizeof(uint32_t); }

// --------------------------------------------------- no-allocation variant --
// The scratch of sfft_dense_topk_noalloc: a file-scope device array with room
// for kNoAllocSpectra spectra (about 1.3 MB), which each device holds from
// module load to process end.  In host code its name is only a stand-in for
// the symbol: kernels get the address hipGetSymbolAddress returns for the
// current device, taken once per device and kept.
constexpr uint32_t kNoAllocSpectra = 64;
constexpr int kNoAllocDevices = 64;
static __device__ __align__(256) uint32_t noalloc_scratch[(size_t)kNoAllocSpectra * kTkStride];

namespace {
std::mutex g_noalloc_mu;
uint32_t* g_noalloc_ptr[kNoAllocDevices] = {};
}  // namespace

uint32_t dense_topk_noalloc_max_count() { return kNoAllocSpectra; }

// The current device's address of noalloc_scratch (looked up on the first
// call on that device).
hipError_t dense_topk_noalloc_scratch(uint32_t** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNoAllocDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_noalloc_ptr[dev] = static_cast<uint32_t*>(p);
    }
    *out = g_noalloc_ptr[dev];
    return hipSuccess;
}

hipError_t launch_dense_topk(const float2* spec, uint64_t n, uint32_t count, uint32_t cap, double scale,
                             double keep_above, uint64_t* out_idx, double* out_val, uint32_t* out_count,
                             uint32_t* scratch, hipStream_t s) {
    // n is a power of two >= 2^10 and nb a power of two <= n / 256, so the
    // chunks tile each spectrum exactly in whole 256-bin tiles
    if (n < 1024 || (n & (n - 1)) || count == 0 || cap == 0) return hipErrorInvalidValue;
    const uint32_t nb = topk_chunks(n);
    const uint64_t chunk = n / nb;
    // keep_above >= 0: keep only bins whose |X|^2 key exceeds that of keep_above
    const uint32_t keep_all = keep_above < 0.0 ? 1u : 0u;
    const float kt = keep_all ? 0.0f : (float)((keep_above / scale) * (keep_above / scale));
    uint32_t KT;
    std::memcpy(&KT, &kt, sizeof(KT));
    hipLaunchKernelGGL(k_topk_init, dim3(count), dim3(kTk), 0, s, scratch, n, cap);
    for (uint32_t pass = 0; pass < 4; ++pass)
        hipLaunchKernelGGL(k_topk_hist, dim3(nb, count), dim3(kTk), 0, s, spec, n, chunk, scratch, pass);
    hipLaunchKernelGGL(k_topk_count, dim3(nb, count), dim3(kTk), 0, s, spec, n, chunk, scratch, keep_all, KT);
    hipLaunchKernelGGL(k_topk_scan, dim3(count), dim3(kTk), 0, s, scratch, nb, cap, keep_all, KT, out_idx, out_val,
                       out_count);
    hipLaunchKernelGGL(k_topk_write, dim3(nb, count), dim3(kTk), 0, s, spec, n, chunk, scratch, cap, keep_all, KT,
                       scale, out_idx, out_val);
    return hipGetLastError();
}

}  // namespace sfft
