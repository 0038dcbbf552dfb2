// Device-side building blocks shared by the kernel sources: precision
// traits, conversions, the SplitMix64 generator, workgroup reductions and
// the fence-free "last workgroup reduces" protocol.
#pragma once

#include "lz_internal.h"

namespace lz {

// Storage type V, SpMV accumulation type A and working-vector type W.
template <int P> struct Tr;
template <> struct Tr<0> { using V = double;   using A = double; using W = double; };
template <> struct Tr<1> { using V = float;    using A = float;  using W = float; };
template <> struct Tr<2> { using V = uint16_t; using A = float;  using W = float; };

__device__ __forceinline__ double to_d(double x) { return x; }
__device__ __forceinline__ double to_d(float x) { return (double)x; }
__device__ __forceinline__ double to_d(uint16_t b) { return (double)__uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ double to_a(double x, double) { return x; }
__device__ __forceinline__ double to_a(float x, double) { return (double)x; }
__device__ __forceinline__ double to_a(uint16_t b, double) { return (double)__uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float to_a(float x, float) { return x; }
__device__ __forceinline__ float to_a(uint16_t b, float) { return __uint_as_float((uint32_t)b << 16); }

// Round-to-nearest-even float -> bfloat16 bits (NaN stays NaN).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
template <class V> __device__ __forceinline__ V from_d(double x);
template <> __device__ __forceinline__ double from_d<double>(double x) { return x; }
template <> __device__ __forceinline__ float from_d<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ uint16_t from_d<uint16_t>(double x) { return f32_to_bf16((float)x); }

// SplitMix64 (Steele, Lea, Flood 2014): output r (0-based) of the stream
// started at `seed`, and the uniform double in [0,1) from its top 53 bits.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t r) {
    uint64_t z = seed + (r + 1ull) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double u01(uint64_t seed, uint64_t r) {
    return (double)(splitmix64(seed, r) >> 11) * (1.0 / 9007199254740992.0);
}

// ------------------------------------------------------------ reductions
template <class T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the threads of a workgroup of `nw` waves; every thread gets it.
template <class T> __device__ __forceinline__ T block_sum(T v, T* sh, int nw = BLOCK / 64) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    T r = sh[0];
    for (int i = 1; i < nw; ++i) r += sh[i];
    return r;
}

// Cross-workgroup data inside one kernel goes through device-coherent
// accesses (they bypass the per-XCD L2 copies), so no device-wide cache
// write-back is needed to publish it.
__device__ __forceinline__ void st_dev(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// True in exactly one workgroup: the last of `count` to arrive.  Every value
// the last workgroup reads from the others must have been written with
// st_dev and is read with ld_dev: each thread waits for its own stores to
// complete before the workgroup takes its ticket.  The ticket is reset for
// the next use.
__device__ __forceinline__ bool last_block(uint32_t* ticket, uint32_t count, int* s_flag) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *s_flag = (t == count - 1u);
    }
    __syncthreads();
    const bool last = *s_flag != 0;
    if (last && threadIdx.x == 0) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return last;
}

// Sum of x[b * stride] over b = first, first + step, ... < nb, in that order
// (device-coherent loads, issued sixteen at a time so that they are in
// flight together).
__device__ __forceinline__ double strided_sum_dev(const double* x, int64_t stride, int first, int step, int nb) {
    double s = 0.0;
    for (int b0 = first; b0 < nb; b0 += 16 * step) {
        double v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = ld_dev(x + (int64_t)min(b0 + i * step, nb - 1) * stride);
#pragma unroll
        for (int i = 0; i < 16; ++i) s += b0 + i * step < nb ? v[i] : 0.0;
    }
    return s;
}

// Sum of x[0..cnt) (device-coherent loads) in a fixed order.
__device__ __forceinline__ double ordered_sum_dev(const double* x, int64_t cnt, double* sh) {
    double s = 0.0;
    int64_t i = threadIdx.x;
    for (; i + 3 * (int64_t)blockDim.x < cnt; i += 4 * (int64_t)blockDim.x) {
        const double a = ld_dev(x + i), b = ld_dev(x + i + blockDim.x), c = ld_dev(x + i + 2 * blockDim.x),
                     d = ld_dev(x + i + 3 * blockDim.x);
        s += ((a + b) + (c + d));
    }
    for (; i < cnt; i += blockDim.x) s += ld_dev(x + i);
    return block_sum(s, sh, blockDim.x / 64);
}

}  // namespace lz
