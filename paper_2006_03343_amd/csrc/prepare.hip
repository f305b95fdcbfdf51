// prepare.hip -- once-per-geometry set-up of the wall-modeled IBM stage.
//
// The paper computes phi and n once (§3.1) and identifies the band points at
// initialisation (§5); this file does that on the GPU:
//   1. node classes of both staggered grids (§3.3 lists) and forcing flags
//      (phi <= 0, eq. f-IB), from the stored phi widened to double and compared
//      against double thresholds, so the result does not depend on the dtype;
//   2. ordered compaction of the band nodes of each grid (block counts, a host
//      scan of the block totals, an in-block scan) -- no atomics, so the record
//      order is the ascending linear index;
//   3. one record per band node: the unit normal (§3.1; central differences on
//      the node's own grid), phi, and the trilinear stencil of the sample point
//      x + (phi_c - phi) n on both node sets (§3.3);
//   4. lists of the kSeg-node segments that hold a solid node (zeroed by the
//      wall-stress pass) or a forced node (forced by the apply pass).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device.h"
#include "geom.h"
#include "ibm_impl.h"

namespace ibm {
namespace {

using namespace geom;

template <typename T>
__global__ void k_classify(const T* __restrict__ pu, const T* __restrict__ pw, long n, double b,
                           double phib, uint8_t* __restrict__ mask, int* __restrict__ bad) {
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double a = (double)pu[q];
    const double w = (double)pw[q];
    if (!isfinite(a) || !isfinite(w)) atomicOr(bad, 1);
    int uvc = a < 0.0 ? 2 : (a <= b ? 1 : 0);
    int wc = w < -phib ? 2 : (w <= phib ? 1 : 0);
    int m = uvc | (wc << 2);
    if (a <= 0.0) m |= 1 << 4;
    if (w <= 0.0) m |= 1 << 5;
    mask[q] = (uint8_t)m;
}

__global__ void k_fmask(const uint8_t* __restrict__ mask, int nx, long rows, int wrow,
                        uint32_t* __restrict__ fmask) {
    long wi = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (wi >= rows * wrow) return;
    long row = wi / wrow;
    int x0 = (int)(wi % wrow) * 16;
    uint32_t bits = 0;
    for (int t = 0; t < 16; ++t) {
        int x = x0 + t;
        if (x < nx) {
            uint32_t m = mask[row * nx + x];
            bits |= ((m >> 4) & 1u) << (2 * t);
            bits |= ((m >> 5) & 1u) << (2 * t + 1);
        }
    }
    fmask[wi] = bits;
}

// Per block of kNodesPerBlock nodes: [uv band, w band, 6 class counts].
__global__ void k_block_counts(const uint8_t* __restrict__ mask, long n, int* __restrict__ bc) {
    __shared__ int lds[8][kCountBlock / 64];
    long q0 = (long)blockIdx.x * kNodesPerBlock + (long)threadIdx.x * kItems;
    int c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int t = 0; t < kItems; ++t) {
        long q = q0 + t;
        if (q < n) {
            int m = mask[q];
            int uvc = m & 3, wc = (m >> 2) & 3;
            c[0] += uvc == 1;
            c[1] += wc == 1;
            c[2 + uvc] += 1;
            c[5 + wc] += 1;
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int i = 0; i < 8; ++i) {
        int x = c[i];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
        if (lane == 0) lds[i][w] = x;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        int s = 0;
        for (int i = 0; i < kCountBlock / 64; ++i) s += lds[threadIdx.x][i];
        bc[(long)blockIdx.x * 8 + threadIdx.x] = s;
    }
}

__global__ void k_compact(const uint8_t* __restrict__ mask, long n, const long* __restrict__ off_uv,
                          const long* __restrict__ off_w, int32_t* __restrict__ q_uv,
                          int32_t* __restrict__ q_w) {
    __shared__ int lds[kCountBlock / 64];
    long q0 = (long)blockIdx.x * kNodesPerBlock + (long)threadIdx.x * kItems;
    int fu = 0, fw = 0;
    uint8_t m[kItems];
    for (int t = 0; t < kItems; ++t) {
        long q = q0 + t;
        m[t] = q < n ? mask[q] : 0;
        fu += (m[t] & 3) == 1;
        fw += ((m[t] >> 2) & 3) == 1;
    }
    int tot;
    int pu = block_exclusive_scan(fu, lds, &tot);
    int pw = block_exclusive_scan(fw, lds, &tot);
    long ou = off_uv[blockIdx.x] + pu;
    long ow = off_w[blockIdx.x] + pw;
    for (int t = 0; t < kItems; ++t) {
        if ((m[t] & 3) == 1) q_uv[ou++] = (int32_t)(q0 + t);
        if (((m[t] >> 2) & 3) == 1) q_w[ow++] = (int32_t)(q0 + t);
    }
}

inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename T>
int prepare_t(ibm_ctx* c, const T* pu, const T* pw, hipStream_t s) {
    const long n = c->n;
    const int nx = c->g.nx, ny = c->g.ny, nz = c->g.nz;
    const long rows = (long)ny * nz;
    const double b = c->p.band_width;
    IBM_HIP(hipMalloc(&c->mask, (size_t)n));
    c->wrow = (nx + 15) / 16;
    IBM_HIP(hipMalloc(&c->fmask, sizeof(uint32_t) * (size_t)rows * c->wrow));
    int* bad = nullptr;
    IBM_HIP(hipMalloc(&bad, sizeof(int)));
    IBM_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_classify<T>, dim3(nblk(n, 256)), dim3(256), 0, s, pu, pw, n, b, 0.5 * b,
                       c->mask, bad);
    hipLaunchKernelGGL(k_fmask, dim3(nblk(rows * c->wrow, 256)), dim3(256), 0, s, c->mask, nx,
                       rows, c->wrow, c->fmask);
    const long nb = (n + kNodesPerBlock - 1) / kNodesPerBlock;
    int* bc = nullptr;
    IBM_HIP(hipMalloc(&bc, sizeof(int) * 8 * (size_t)nb));
    hipLaunchKernelGGL(k_block_counts, dim3((unsigned)nb), dim3(kCountBlock), 0, s, c->mask, n, bc);
    IBM_HIP(hipGetLastError());
    std::vector<int> hbc(8 * (size_t)nb);
    int hbad = 0;
    IBM_HIP(hipMemcpyAsync(hbc.data(), bc, sizeof(int) * 8 * (size_t)nb, hipMemcpyDeviceToHost, s));
    IBM_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    (void)hipFree(bad);
    if (hbad) {
        (void)hipFree(bc);
        return fail(IBM_E_RANGE, "levelset_prepare: phi_uv or phi_w holds a non-finite value");
    }
    std::vector<long> off_uv(nb), off_w(nb);
    long tu = 0, tw = 0;
    for (int i = 0; i < 6; ++i) c->counts[i] = 0;
    for (long b_ = 0; b_ < nb; ++b_) {
        off_uv[b_] = tu;
        off_w[b_] = tw;
        tu += hbc[8 * b_ + 0];
        tw += hbc[8 * b_ + 1];
        for (int i = 0; i < 6; ++i) c->counts[i] += hbc[8 * b_ + 2 + i];
    }
    int rc = alloc_records(c->rec[0], tu, sizeof(T));
    if (rc) return rc;
    rc = alloc_records(c->rec[1], tw, sizeof(T));
    if (rc) return rc;
    long* doff = nullptr;
    IBM_HIP(hipMalloc(&doff, sizeof(long) * 2 * (size_t)nb));
    IBM_HIP(hipMemcpyAsync(doff, off_uv.data(), sizeof(long) * nb, hipMemcpyHostToDevice, s));
    IBM_HIP(hipMemcpyAsync(doff + nb, off_w.data(), sizeof(long) * nb, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_compact, dim3((unsigned)nb), dim3(kCountBlock), 0, s, c->mask, n, doff,
                       doff + nb, c->rec[0].q, c->rec[1].q);
    GeomArgs ga{nx, ny, nz, c->g.dx, c->g.dy, c->g.dz, c->p.phi_c};
    const bool mixed = c->precision == IBM_PREC_MIXED;
    for (int kind = 0; kind < 2; ++kind) {
        Records& R = c->rec[kind];
        if (R.n == 0) continue;
        RecOut o{R.q, R.base, R.sx, R.sy, R.ku, R.kw, R.nrm[0], R.nrm[1], R.nrm[2], R.phi,
                 R.fx, R.fy, R.fzu, R.fzw};
        const T* ph = kind == 0 ? pu : pw;
        if (mixed)
            hipLaunchKernelGGL((k_records<T, true>), dim3(nblk(R.n, 256)), dim3(256), 0, s, ph,
                               kind, R.n, o, ga);
        else
            hipLaunchKernelGGL((k_records<T, false>), dim3(nblk(R.n, 256)), dim3(256), 0, s, ph,
                               kind, R.n, o, ga);
    }
    // segments with solid nodes (zeroed by wall_stress) and with forced nodes
    // (forced by apply)
    const long nseg = (n + kSeg - 1) / kSeg;
    uint8_t* dflags = nullptr;
    IBM_HIP(hipMalloc(&dflags, (size_t)nseg));
    hipLaunchKernelGGL(k_seg_flags, dim3((unsigned)nseg), dim3(256), 0, s, c->mask, n, dflags);
    IBM_HIP(hipGetLastError());
    std::vector<uint8_t> hf(nseg);
    IBM_HIP(hipMemcpyAsync(hf.data(), dflags, (size_t)nseg, hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    (void)hipFree(dflags);
    std::vector<Seg> zs, fs;
    for (long i = 0; i < nseg; ++i) {
        const int32_t q = (int32_t)(i * kSeg);
        const int32_t len = (int32_t)std::min<long>(kSeg, n - i * kSeg);
        if (hf[i] & 3) zs.push_back(Seg{q, len, hf[i] & 3, 0});
        if (hf[i] & 12) fs.push_back(Seg{q, len, (hf[i] >> 2) & 3, 0});
    }
    c->nzsegs = (long)zs.size();
    c->nfsegs = (long)fs.size();
    IBM_HIP(hipMalloc(&c->zsegs, sizeof(Seg) * std::max<size_t>(zs.size(), 1)));
    IBM_HIP(hipMalloc(&c->fsegs, sizeof(Seg) * std::max<size_t>(fs.size(), 1)));
    if (!zs.empty())
        IBM_HIP(hipMemcpy(c->zsegs, zs.data(), sizeof(Seg) * zs.size(), hipMemcpyHostToDevice));
    if (!fs.empty())
        IBM_HIP(hipMemcpy(c->fsegs, fs.data(), sizeof(Seg) * fs.size(), hipMemcpyHostToDevice));
    (void)hipFree(doff);
    (void)hipFree(bc);
    return IBM_OK;
}

}  // namespace

void free_prepared(ibm_ctx* c) {
    (void)hipFree(c->mask);
    c->mask = nullptr;
    (void)hipFree(c->fmask);
    c->fmask = nullptr;
    for (int k = 0; k < 2; ++k) {
        (void)hipFree(c->rec[k].buf);
        c->rec[k] = Records();
    }
    (void)hipFree(c->zsegs);
    c->zsegs = nullptr;
    c->nzsegs = 0;
    (void)hipFree(c->fsegs);
    c->fsegs = nullptr;
    c->nfsegs = 0;
    free_adjoint(c);
    free_chester(c);
    c->prepared = false;
}

int prepare(ibm_ctx* c, const void* phi_uv, const void* phi_w, hipStream_t s) {
    free_prepared(c);
    int rc = c->dtype == IBM_F64 ? prepare_t<double>(c, (const double*)phi_uv, (const double*)phi_w, s)
                                 : prepare_t<float>(c, (const float*)phi_uv, (const float*)phi_w, s);
    if (rc != IBM_OK) {
        free_prepared(c);
        return rc;
    }
    c->prepared = true;
    return IBM_OK;
}

}  // namespace ibm
