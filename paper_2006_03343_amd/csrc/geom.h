// geom.h -- once-per-geometry helpers shared by the simplified method's
// set-up (prepare.hip) and that of Chester et al.'s original (chester.hip):
// ordered compaction scans, the per-segment class flags and the band-record
// builder (unit normal of §3.1 by central differences on the node's own grid,
// and the trilinear stencil of a point at a given distance from the surface
// along the normal on both node sets, §3.3).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device.h"
#include "ibm_impl.h"

namespace ibm {
namespace geom {
namespace {   // device code: each including source keeps its own copy

constexpr int kItems = 8;                    // nodes per thread in the count/compact pass
constexpr int kCountBlock = 256;
constexpr int kNodesPerBlock = kItems * kCountBlock;

__device__ inline int block_exclusive_scan(int x, int* lds, int* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) lds[w] = inc;
    __syncthreads();
    int pre = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        if (i < w) pre += lds[i];
        tot += lds[i];
    }
    __syncthreads();
    *total = tot;
    return pre + inc - x;
}

// Per segment of kSeg linear indices: bit 0 some uv node solid (class code 2
// or 3), bit 1 some w node solid, bit 2 some uv node forced, bit 3 some w node forced.
__global__ void __launch_bounds__(256) k_seg_flags(const uint8_t* __restrict__ mask, long n,
                                                   uint8_t* __restrict__ flags) {
    __shared__ int acc;
    if (threadIdx.x == 0) acc = 0;
    __syncthreads();
    const long q0 = (long)blockIdx.x * kSeg;
    int bits = 0;
    for (int t = threadIdx.x; t < kSeg; t += blockDim.x) {
        if (q0 + t >= n) break;
        const int m = mask[q0 + t];
        bits |= ((m & 3) >= 2 ? 1 : 0) | (((m >> 2) & 3) >= 2 ? 2 : 0) | (((m >> 4) & 3) << 2);
    }
    if (bits) atomicOr(&acc, bits);
    __syncthreads();
    if (threadIdx.x == 0) flags[blockIdx.x] = (uint8_t)acc;
}

struct RecOut {
    int32_t *q, *base, *sx, *sy, *ku, *kw;
    void *nx, *ny, *nz, *phi, *fx, *fy, *fzu, *fzw;
};

struct GeomArgs {
    int nx, ny, nz;
    double dx, dy, dz;
    double phi_c;
};

// Lower stencil index and fraction of the vertical index coordinate k + t,
// clamped to [0, nz-1].  Splitting the small offset t keeps the fraction
// exact to the precision of t even on tall grids.
template <typename T>
__device__ inline void vsplit(int k, T t, int nz, int32_t* k0, T* f) {
    T fl = floor(t);
    int kk = k + (int)fl;
    T fr = t - fl;
    if (kk >= nz - 1) {
        kk = nz - 1;
        fr = T(0);
    }
    if (kk < 0) {
        kk = 0;
        fr = T(0);
    }
    *k0 = kk;
    *f = fr;
}

template <typename T>
__device__ inline void hsplit(int i, T t, int n, int32_t* i0, T* f) {
    T fl = floor(t);
    long ii = (long)i + (long)fl;
    *f = t - fl;
    *i0 = (int32_t)pmodl(ii, n);
}

template <typename T, bool MIXED>
__global__ void k_records(const T* __restrict__ phi, int kind, long nrec, RecOut o, GeomArgs ga) {
    long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrec) return;
    const int nx = ga.nx, ny = ga.ny, nz = ga.nz;
    const long plane = (long)nx * ny;
    const long q = o.q[r];
    const int i = (int)(q % nx);
    const int j = (int)((q / nx) % ny);
    const int k = (int)(q / plane);
    const long row = q - i;
    const long col = q - (long)j * nx;
    // neighbours on the node's own grid: periodic in x and y
    const T pxp = phi[row + pmodl(i + 1, nx)], pxm = phi[row + pmodl(i - 1, nx)];
    const T pyp = phi[col + pmodl(j + 1, ny) * nx], pym = phi[col + pmodl(j - 1, ny) * nx];
    T pzp = phi[q], pzm = phi[q];
    T hz = T(2);
    if (nz == 1) {
        hz = T(1);
    } else if (k == 0) {
        pzp = phi[q + plane];
        hz = T(1);
    } else if (k == nz - 1) {
        pzm = phi[q - plane];
        hz = T(1);
    } else {
        pzp = phi[q + plane];
        pzm = phi[q - plane];
    }
    T gx = (pxp - pxm) / (T(2) * T(ga.dx));
    T gy = (pyp - pym) / (T(2) * T(ga.dy));
    T gz = (pzp - pzm) / (hz * T(ga.dz));
    T m2 = gx * gx + gy * gy + gz * gz;
    T n0, n1, n2;
    if (MIXED && m2 < T(0.25)) {
        // small |grad phi|: difference and normalise in double (the float
        // differences of float values are exact in double)
        double dgx = ((double)pxp - (double)pxm) / (2.0 * ga.dx);
        double dgy = ((double)pyp - (double)pym) / (2.0 * ga.dy);
        double dgz = ((double)pzp - (double)pzm) / ((double)hz * ga.dz);
        double mag = sqrt(dgx * dgx + dgy * dgy + dgz * dgz);
        if (mag == 0.0) {
            n0 = T(0); n1 = T(0); n2 = T(1);
        } else {
            n0 = (T)(dgx / mag); n1 = (T)(dgy / mag); n2 = (T)(dgz / mag);
        }
    } else if (m2 == T(0)) {
        n0 = T(0); n1 = T(0); n2 = T(1);
    } else {
        T mag = sqrt(m2);
        n0 = gx / mag; n1 = gy / mag; n2 = gz / mag;
    }
    // sample point offset from the node, in cells
    const T shift = T(ga.phi_c) - phi[q];
    const T tx = shift * n0 / T(ga.dx);
    const T ty = shift * n1 / T(ga.dy);
    const T tz = shift * n2 / T(ga.dz);
    int32_t i0, j0, ku, kw;
    T fx, fy, fzu, fzw;
    hsplit<T>(i, tx, nx, &i0, &fx);
    hsplit<T>(j, ty, ny, &j0, &fy);
    // node heights in index units: uv node k+1/2, w node k; uv index = z/dz - 1/2
    const T tu = kind == IBM_GRID_UV ? tz : tz - T(0.5);
    const T tw = kind == IBM_GRID_UV ? tz + T(0.5) : tz;
    vsplit<T>(k, tu, nz, &ku, &fzu);
    vsplit<T>(k, tw, nz, &kw, &fzw);
    o.base[r] = j0 * nx + i0;
    o.sx[r] = (i0 + 1 == nx) ? 1 - nx : 1;
    o.sy[r] = (j0 + 1 == ny) ? (1 - ny) * nx : nx;
    o.ku[r] = ku;
    o.kw[r] = kw;
    ((T*)o.nx)[r] = n0;
    ((T*)o.ny)[r] = n1;
    ((T*)o.nz)[r] = n2;
    ((T*)o.phi)[r] = phi[q];
    ((T*)o.fx)[r] = fx;
    ((T*)o.fy)[r] = fy;
    ((T*)o.fzu)[r] = fzu;
    ((T*)o.fzw)[r] = fzw;
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

inline int alloc_records(Records& R, long n, size_t ts) {
    R.n = n;
    size_t ib = align256(sizeof(int32_t) * (size_t)std::max<long>(n, 1));
    size_t tb = align256(ts * (size_t)std::max<long>(n, 1));
    size_t total = 6 * ib + 8 * tb;
    IBM_HIP(hipMalloc(&R.buf, total));
    char* p = (char*)R.buf;
    int32_t** ints[6] = {&R.q, &R.base, &R.sx, &R.sy, &R.ku, &R.kw};
    for (int i = 0; i < 6; ++i) {
        *ints[i] = (int32_t*)p;
        p += ib;
    }
    void** ts_[8] = {&R.nrm[0], &R.nrm[1], &R.nrm[2], &R.phi, &R.fx, &R.fy, &R.fzu, &R.fzw};
    for (int i = 0; i < 8; ++i) {
        *ts_[i] = p;
        p += tb;
    }
    return IBM_OK;
}

}  // namespace
}  // namespace geom
}  // namespace ibm
