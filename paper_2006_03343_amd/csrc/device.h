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

// A raw buffer resource (stride 0, no range limit) whose base is a
// wave-uniform pointer: loads through it take the lane's byte offset in a
// vector register and a uniform byte offset in a scalar register, so a wave
// that marches through rows and planes adds offsets in scalar registers only.
// Offsets are 32-bit: base + offsets must stay within 4 GiB of the base.
typedef __amdgpu_buffer_rsrc_t Rsrc;

__device__ inline Rsrc buffer_rsrc(const void* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, -1, 0x00020000);
}

template <typename T, int VX>
__device__ inline Vec<T, VX> bload(Rsrc r, unsigned lane_off, unsigned uniform_off) {
    constexpr int B = (int)sizeof(T) * VX;
    static_assert(B == 4 || B == 8 || B == 16, "bload: 4, 8 or 16 bytes per lane");
    Vec<T, VX> out;
    if constexpr (B == 4) {
        const auto x = __builtin_amdgcn_raw_buffer_load_b32(r, (int)lane_off, (int)uniform_off, 0);
        __builtin_memcpy(out.v, &x, 4);
    } else if constexpr (B == 8) {
        const auto x = __builtin_amdgcn_raw_buffer_load_b64(r, (int)lane_off, (int)uniform_off, 0);
        __builtin_memcpy(out.v, &x, 8);
    } else {
        const auto x = __builtin_amdgcn_raw_buffer_load_b128(r, (int)lane_off, (int)uniform_off, 0);
        __builtin_memcpy(out.v, &x, 16);
    }
    return out;
}

__device__ inline uint32_t bload_u8(Rsrc r, unsigned lane_off, unsigned uniform_off) {
    return __builtin_amdgcn_raw_buffer_load_b8(r, (int)lane_off, (int)uniform_off, 0);
}

// n / d and sqrt(x) for the eddy viscosity: in float the hardware's reciprocal
// and square root (1 ulp each, a few instructions fewer than the correctly
// rounded sequences), in double the correctly rounded operations.
__device__ inline float quot_fast(float n, float d) { return n * __builtin_amdgcn_rcpf(d); }
__device__ inline double quot_fast(double n, double d) { return n / d; }
__device__ inline float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double sqrt_fast(double x) { return __builtin_sqrt(x); }

// XCD-aware block order.  Blocks are dealt round-robin over the 8 XCDs
// (block b on XCD b % 8); block b takes logical block (b % 8) * per_xcd + b / 8,
// so each XCD runs a contiguous range of logical blocks and neighbours share
// its L2.  The grid holds 8 * per_xcd blocks; -1 for the padding blocks.
__device__ inline int xcd_block(int nblocks) {
    const int per_xcd = (nblocks + 7) >> 3;
    const int lb = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
    return lb < nblocks ? lb : -1;
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
