// device.h -- small device helpers shared by the kernels of this library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ibm {

__host__ __device__ inline long pmodl(long a, long n) {
    long r = a % n;
    return r < 0 ? r + n : r;
}

// Vector of VX consecutive elements held by one lane, moved with one load.
template <typename T, int VX>
struct Vec {
    T v[VX];
};

template <typename T, int VX>
__device__ inline Vec<T, VX> vload(const T* p) {
    Vec<T, VX> r;
    if constexpr (sizeof(T) * VX == 16) {
        const uint4 raw = *reinterpret_cast<const uint4*>(p);
        __builtin_memcpy(r.v, &raw, 16);
    } else if constexpr (sizeof(T) * VX == 8) {
        const uint2 raw = *reinterpret_cast<const uint2*>(p);
        __builtin_memcpy(r.v, &raw, 8);
    } else {
#pragma unroll
        for (int e = 0; e < VX; ++e) r.v[e] = p[e];
    }
    return r;
}

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// Streaming (non-temporal) store of a lane's vector: the divergence is written
// once and not read again by this pass.
template <typename T, int VX>
__device__ inline void vstore_nt(T* p, const Vec<T, VX>& r) {
    if constexpr (sizeof(T) * VX == 16) {
        u32x4 raw;
        __builtin_memcpy(&raw, r.v, 16);
        __builtin_nontemporal_store(raw, reinterpret_cast<u32x4*>(p));
    } else if constexpr (sizeof(T) * VX == 8) {
        u32x2 raw;
        __builtin_memcpy(&raw, r.v, 8);
        __builtin_nontemporal_store(raw, reinterpret_cast<u32x2*>(p));
    } else {
#pragma unroll
        for (int e = 0; e < VX; ++e) __builtin_nontemporal_store(r.v[e], p + e);
    }
}

template <typename T, int VX>
__device__ inline Vec<T, VX> vzero() {
    Vec<T, VX> r;
#pragma unroll
    for (int e = 0; e < VX; ++e) r.v[e] = T(0);
    return r;
}

// Butterfly sum / max over the 64 lanes of a wave (fixed order: deterministic).
__device__ inline double wave_sum(double x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

__device__ inline double wave_max(double x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x = fmax(x, __shfl_xor(x, m, 64));
    return x;
}

}  // namespace ibm
