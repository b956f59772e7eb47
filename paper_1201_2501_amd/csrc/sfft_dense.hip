// Dense fallback of the serving runtime: after a full-length FFT of each
// signal, keep the `cap` bins of largest magnitude (ties: the smaller index),
// in ascending index order.  Used where the flat window would cover the whole
// signal (w >= n), so the sparse method has nothing to save.
//
// One 1024-thread workgroup per spectrum.  Radix select on the FP32 bit
// pattern of |X_f|^2 (non-negative floats order as unsigned integers): four
// 8-bit passes find the key T of the cap-th largest bin and how many bins
// equal to T are taken; one pass in index order with block scans then writes
// the kept bins in ascending index order.
#include "sfft_device.hpp"

namespace sfft {

namespace {

constexpr uint32_t kDense = 1024;

__device__ __forceinline__ uint32_t mag_bits(float2 v) { return __float_as_uint(v.x * v.x + v.y * v.y); }

// Exclusive prefix of one flag per thread over the block; returns the total.
__device__ uint32_t block_scan_1024(uint32_t v, uint32_t* wsum, uint32_t* prefix) {
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
    for (uint32_t w = 0; w < kDense / 64; ++w) {
        const uint32_t c = wsum[w];
        before += w < wave ? c : 0u;
        total += c;
    }
    *prefix = before + inc - v;
    return total;
}

__global__ void __launch_bounds__(kDense) k_dense_topk(const float2* __restrict__ spec, uint64_t n, uint32_t cap,
                                                       double scale, double keep_above, uint64_t* out_idx,
                                                       double* out_val, uint32_t* out_count) {
    __shared__ uint32_t hist[256];
    __shared__ uint32_t wsum[kDense / 64];
    __shared__ uint32_t sel[2];   // key prefix, bins equal to T still to take
    const uint32_t tid = threadIdx.x;
    const uint32_t sig = blockIdx.x;
    const float2* x = spec + (uint64_t)sig * n;
    uint64_t* oi = out_idx + (uint64_t)sig * cap;
    double* ov = out_val + (uint64_t)sig * cap * 2;
    const bool all = (uint64_t)cap >= n;
    uint32_t T = 0, take_eq = 0;
    if (!all) {
        uint32_t prefix = 0, mask = 0, need = cap;   // need: rank of T among keys matching prefix, from the top
        for (int pass = 0; pass < 4; ++pass) {
            const uint32_t shift = 24 - 8 * pass;
            for (uint32_t d = tid; d < 256; d += kDense) hist[d] = 0;
            __syncthreads();
            for (uint64_t f = tid; f < n; f += kDense) {
                const uint32_t k = mag_bits(x[f]);
                if ((k & mask) == prefix) atomicAdd(&hist[(k >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (tid == 0) {
                uint32_t acc = 0, digit = 0;
                for (int d = 255; d >= 0; --d) {
                    if (acc + hist[d] >= need) {
                        digit = (uint32_t)d;
                        break;
                    }
                    acc += hist[d];
                }
                sel[0] = prefix | (digit << shift);
                sel[1] = need - acc;
            }
            __syncthreads();
            prefix = sel[0];
            need = sel[1];
            mask |= 255u << shift;
        }
        T = prefix;
        take_eq = need;   // bins with key == T to take, smallest indices first
    }
    uint32_t written = 0, ties = 0;
    for (uint64_t base = 0; base < n; base += kDense) {
        const uint64_t f = base + tid;
        float2 v = make_float2(0.f, 0.f);
        uint32_t k = 0;
        if (f < n) {
            v = x[f];
            k = mag_bits(v);
        }
        const bool in = f < n;
        const bool gt = in && (all || k > T);
        const bool eq = in && !all && k == T;
        uint32_t tie_pre;
        const uint32_t tie_tot = block_scan_1024(eq ? 1u : 0u, wsum, &tie_pre);
        const bool chosen = gt || (eq && ties + tie_pre < take_eq);
        const double vr = (double)v.x * scale, vi = (double)v.y * scale;
        const bool keep = chosen && sqrt(vr * vr + vi * vi) > keep_above;
        uint32_t pos;
        const uint32_t kept = block_scan_1024(keep ? 1u : 0u, wsum, &pos);
        if (keep) {
            oi[written + pos] = f;
            ov[2 * (written + pos)] = vr;
            ov[2 * (written + pos) + 1] = vi;
        }
        written += kept;
        ties += tie_tot;
    }
    for (uint32_t q = written + tid; q < cap; q += kDense) {
        oi[q] = 0;
        ov[2 * q] = 0.0;
        ov[2 * q + 1] = 0.0;
    }
    if (tid == 0) out_count[sig] = written;
}

}  // namespace

hipError_t launch_dense_topk(const float2* spec, uint64_t n, uint32_t count, uint32_t cap, double scale,
                             double keep_above, uint64_t* out_idx, double* out_val, uint32_t* out_count,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_dense_topk, dim3(count), dim3(kDense), 0, s, spec, n, cap, scale, keep_above, out_idx,
                       out_val, out_count);
    return hipGetLastError();
}

}  // namespace sfft
