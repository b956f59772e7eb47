// Device helpers shared by the HIP kernels: complex arithmetic, exact
// roots of unity, bit reversal, and block-wide sort/scan primitives.
#pragma once

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

// ------------------------------------------------------------------------
// Block-wide helpers for the decode kernels.

// Bitonic sort (ascending) of N = power-of-two 64-bit keys in LDS by a
// block of NT threads.
template <uint32_t NT = kThreads>
__device__ static void bitonic_sort_u64(uint64_t* key, uint32_t N) {
    for (uint32_t size = 2; size <= N; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (uint32_t t = threadIdx.x; t < N / 2; t += NT) {
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

// Exclusive prefix sum of one value per thread of a block of NT threads;
// returns the block total.
template <uint32_t NT = kThreads>
__device__ static uint32_t block_exclusive_scan(uint32_t v, uint32_t* scratch, uint32_t* out_prefix) {
    const uint32_t tid = threadIdx.x;
    __syncthreads();
    scratch[tid] = v;
    __syncthreads();
    for (uint32_t off = 1; off < NT; off <<= 1) {
        const uint32_t add = tid >= off ? scratch[tid - off] : 0u;
        __syncthreads();
        scratch[tid] += add;
        __syncthreads();
    }
    *out_prefix = scratch[tid] - v;
    const uint32_t total = scratch[NT - 1];
    __syncthreads();
    return total;
}

template <class K>
static inline hipError_t allow_lds(K kernel, size_t lds) {
    if (lds <= 64 * 1024) return hipSuccess;
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

}  // namespace sfft
