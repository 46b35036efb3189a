// sv_device.h -- device helpers shared by the kernels of libsv.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sv {

constexpr int kBlock = 256;   // threads per workgroup of the sweep kernels (4 wave64)

// Insert a 0 bit at each position of pos[0..np) (ascending) into g: maps a
// compact index over the free bits to an amplitude index whose bits at pos
// are 0.
__device__ __forceinline__ uint64_t insert_zeros(uint64_t g, const int* pos, int np)
{
    for (int i = 0; i < np; ++i) {
        const uint64_t lo = g & ((1ull << pos[i]) - 1ull);
        g = ((g >> pos[i]) << (pos[i] + 1)) | lo;
    }
    return g;
}

// Load of a table entry at a uniform address through the scalar cache: for
// tables that stay read-only while the kernel runs (launch tables, Pauli
// terms), read as constant memory, a word at a time.
template <class T>
__device__ __forceinline__ T ld_const(const T* p)
{
    static_assert(sizeof(T) % 4 == 0, "whole words");
    typedef const __attribute__((address_space(4))) uint32_t cword;
    const cword* q = (const cword*)p;
    uint32_t w[sizeof(T) / 4];
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = q[i];
    return __builtin_bit_cast(T, w);
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// c + a * b
__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c)
{
    return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}

// Streaming (non-temporal) 16- and 8-byte accesses: every amplitude of a
// sweep is touched once, so there is nothing to keep in the caches. Only
// worth it when every 128-byte line a kernel writes is written whole: a
// partially written line that bypasses the cache is merged in memory, which
// costs far more than the cached path. The NT template flag selects.
typedef float sv_v4f __attribute__((ext_vector_type(4)));
typedef float sv_v2f __attribute__((ext_vector_type(2)));

template <bool NT = true>
__device__ __forceinline__ float4 ld4(const float2* p)
{
    if constexpr (NT) {
        const sv_v4f v = __builtin_nontemporal_load(reinterpret_cast<const sv_v4f*>(p));
        return make_float4(v.x, v.y, v.z, v.w);
    } else {
        return *reinterpret_cast<const float4*>(p);
    }
}

template <bool NT = true>
__device__ __forceinline__ void st4(float2* p, float4 x)
{
    if constexpr (NT) {
        const sv_v4f v = {x.x, x.y, x.z, x.w};
        __builtin_nontemporal_store(v, reinterpret_cast<sv_v4f*>(p));
    } else {
        *reinterpret_cast<float4*>(p) = x;
    }
}

template <bool NT = true>
__device__ __forceinline__ float2 ld2(const float2* p)
{
    if constexpr (NT) {
        const sv_v2f v = __builtin_nontemporal_load(reinterpret_cast<const sv_v2f*>(p));
        return make_float2(v.x, v.y);
    } else {
        return *p;
    }
}

template <bool NT = true>
__device__ __forceinline__ void st2(float2* p, float2 x)
{
    if constexpr (NT) {
        const sv_v2f v = {x.x, x.y};
        __builtin_nontemporal_store(v, reinterpret_cast<sv_v2f*>(p));
    } else {
        *p = x;
    }
}

// Lowest qubit whose runs of consecutive amplitudes are written whole by a
// sweep that skips positions below it: runs of 2^4 amplitudes = 128 bytes.
constexpr int kFullLineQubit = 4;

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8). Renumbering so that each XCD sweeps one contiguous eighth of the
// block range keeps every XCD's concurrent accesses close together in
// memory (measured ~10% faster sweeps at large strides). A bijection only
// when the block count is a multiple of 8; otherwise the identity.
__device__ __forceinline__ uint64_t xcd_block(uint64_t b, uint64_t nb)
{
    return (nb & 7) ? b : (b & 7) * (nb >> 3) + (b >> 3);
}

__device__ __forceinline__ float2 lo2(float4 v) { return make_float2(v.x, v.y); }
__device__ __forceinline__ float2 hi2(float4 v) { return make_float2(v.z, v.w); }
__device__ __forceinline__ float4 pack4(float2 a, float2 b) { return make_float4(a.x, a.y, b.x, b.y); }

// Sum NV doubles over a 256-thread block; the result is valid in thread 0.
// The order of additions is fixed, so the result is bitwise reproducible.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV])
{
    __shared__ double sh[kBlock / 64][NV];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] += __shfl_xor(v[i], off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) sh[w][i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double s = sh[0][i];
#pragma unroll
            for (int j = 1; j < kBlock / 64; ++j) s += sh[j][i];
            v[i] = s;
        }
}

}  // namespace sv
