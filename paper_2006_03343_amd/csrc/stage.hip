// stage.hip -- per-case launches of the stage kernels (device code in
// kernels.h): the wall-stress pass with its statistics, the dense pass with
// forcing and drag, and the fixed-order finalize of the reductions; and the
// one-call stage, which runs both passes and sums both sets of slots in one
// launch.
#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace ibm {
namespace {

template <typename T, bool MIXED, bool HAS_LZ>
__global__ void __launch_bounds__(kBandBlock) k_wall_stress(WSArgs<T> a) {
    ws_block<T, MIXED, HAS_LZ>(a, blockIdx.x);
}

// Fixed-order reduction of per-slot partials (one block).
__global__ void __launch_bounds__(256) k_finalize(const double* __restrict__ p, long nslots, int nc,
                                                   unsigned maxmask, double scale,
                                                   double* __restrict__ out) {
    finalize_slots(p, nslots, nc, maxmask, scale, out);
}

// The first 8 * per_xcd blocks own wave-tiles, taken in an XCD-aware order
// (the dispatcher deals blocks to the 8 XCDs round-robin, so block b runs on
// XCD b % 8, and consecutive tiles -- which share halos -- are given to the
// same XCD's L2).  The blocks after them force the segments holding nodes with
// phi <= 0.  Tiles come first so that they spread evenly over an idle GPU:
// placed behind short blocks of another role they were dispatched as those
// retired and piled onto the CUs that freed first.
template <typename T, typename Acc, int VX, int TY>
__global__ void __launch_bounds__(256) k_apply(ApplyArgs<T> a) {
    const int ntb = 8 * a.per_xcd;
    if ((int)blockIdx.x >= ntb) {
        // quarters of the forcing segments, so a short launch is not left
        // waiting on a few blocks that each force a whole segment
        constexpr int kPiece = kSeg / 4;
        for (long it = blockIdx.x - ntb; it < 4 * a.nfsegs; it += a.nfblocks) {
            const Seg sg = a.fsegs[it >> 2];
            const int off = (int)(it & 3) * kPiece;
            if (off < sg.len)
                force_seg<T>(a, Seg{sg.q + off, min(kPiece, sg.len - off), 0, 0}, threadIdx.x,
                             blockDim.x);
        }
        return;
    }
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpb = blockDim.x >> 6;
    const int lb = (blockIdx.x & 7) * a.per_xcd + (blockIdx.x >> 3);
    const long tile = (long)lb * wpb + wv;
    if (lb < a.nblocks && tile < a.ntiles) apply_tile<T, Acc, VX, TY>(a, tile, lane);
}

template <typename T>
int wall_stress_t(ibm_ctx* c, const T* u, const T* v, const T* w, double z0, const T* log_z0,
                  void* const tau[6], double* stats, hipStream_t s, bool finalize = true) {
    WSArgs<T> a = make_ws_args<T>(c, u, v, w, z0, log_z0, tau, stats);
    if (c->ws_cap < 4L * a.nb_band) return fail(IBM_E_STATE, "wall_stress: reduction slots not sized");
    const unsigned grid = (unsigned)(a.nb_band + c->nzsegs);
    const bool mixed = c->precision == IBM_PREC_MIXED;
    if (mixed && log_z0)
        hipLaunchKernelGGL((k_wall_stress<T, true, true>), dim3(grid), dim3(kBandBlock), 0, s, a);
    else if (mixed)
        hipLaunchKernelGGL((k_wall_stress<T, true, false>), dim3(grid), dim3(kBandBlock), 0, s, a);
    else if (log_z0)
        hipLaunchKernelGGL((k_wall_stress<T, false, true>), dim3(grid), dim3(kBandBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_wall_stress<T, false, false>), dim3(grid), dim3(kBandBlock), 0, s, a);
    if (stats && finalize)
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, (const double*)a.partials,
                           (long)a.nb_band, 4, 1u << 2, 1.0, stats);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

// The slot sums of one stage pass in one launch of two blocks, which run side
// by side: block 0 the wall stress's band statistics (4 per band block),
// block 1 the dense pass's drag (3 per tile).  Each is k_finalize's sum.
__global__ void __launch_bounds__(256) k_finalize_stage(const double* __restrict__ ws, long nws,
                                                         double* __restrict__ stats,
                                                         const double* __restrict__ ap, long nap,
                                                         double dv, double* __restrict__ drag) {
    if (blockIdx.x == 0) {
        if (stats) finalize_slots(ws, nws, 4, 1u << 2, 1.0, stats);
    } else if (drag) {
        finalize_slots(ap, nap, 3, 0u, dv, drag);
    }
}

template <typename T, typename Acc, int VX, int TY>
void launch_apply_k(const ApplyArgs<T>& a, unsigned grid, unsigned block, hipStream_t s) {
    hipLaunchKernelGGL((k_apply<T, Acc, VX, TY>), dim3(grid), dim3(block), 0, s, a);
}

template <typename T, typename Acc, int VX>
bool dispatch_ty(const ApplyArgs<T>& a, int ty, unsigned grid, unsigned block, hipStream_t s) {
    switch (ty) {
        case 1: launch_apply_k<T, Acc, VX, 1>(a, grid, block, s); return true;
        case 2: launch_apply_k<T, Acc, VX, 2>(a, grid, block, s); return true;
        case 4: launch_apply_k<T, Acc, VX, 4>(a, grid, block, s); return true;
        case 8: launch_apply_k<T, Acc, VX, 8>(a, grid, block, s); return true;
        default: return false;
    }
}

template <typename T, typename Acc>
bool dispatch_vx(const ApplyArgs<T>& a, int vx, int ty, unsigned grid, unsigned block,
                 hipStream_t s) {
    switch (vx) {
        case 1: return dispatch_ty<T, Acc, 1>(a, ty, grid, block, s);
        case 2: return dispatch_ty<T, Acc, 2>(a, ty, grid, block, s);
        case 4:
            if constexpr (sizeof(T) == 4) return dispatch_ty<T, Acc, 4>(a, ty, grid, block, s);
            return false;
        default: return false;
    }
}

template <typename T>
int apply_t(ibm_ctx* c, const TileCfg& cfg, const void* const tau[6], void* const ustar[3],
            const void* const gradp[3], double dt, void* const div[3], double* drag,
            hipStream_t s, double* partials, bool finalize = true) {
    ApplyArgs<T> a = make_apply_args<T>(c, cfg, tau, ustar, gradp, dt, div, drag);
    if (partials)
        a.partials = partials;   // the caller's slots, of at least 3 * ntiles doubles
    else if (c->ap_cap < 3 * a.ntiles)
        return fail(IBM_E_STATE, "apply: reduction slots not sized");
    a.nfblocks = (int)std::min<long>((4 * c->nfsegs + 7) / 8 * 8, 2048);
    const unsigned grid = (unsigned)(a.nfblocks + 8 * a.per_xcd);
    const unsigned block = (unsigned)(64 * cfg.wpb);
    bool ok;
    if (c->precision == IBM_PREC_MIXED || sizeof(T) == 8)
        ok = dispatch_vx<T, double>(a, cfg.vx, cfg.ty, grid, block, s);
    else
        ok = dispatch_vx<T, float>(a, cfg.vx, cfg.ty, grid, block, s);
    if (!ok) return fail(IBM_E_ARG, "apply: unsupported tile shape vx=%d ty=%d", cfg.vx, cfg.ty);
    if (drag && finalize)
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, (const double*)a.partials,
                           a.ntiles, 3, 0u, a.dv, drag);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

// One stage pass: the wall-stress kernel, the dense pass, and one launch
// for both slot sums (the same slots and order as the two calls, so the
// results are theirs bit for bit).
template <typename T>
int stage_t(ibm_ctx* c, const TileCfg& cfg, const T* u, const T* v, const T* w, double z0,
            const T* log_z0, void* const tau[6], void* const ustar[3], const void* const gradp[3],
            double dt, void* const div[3], double* stats, double* drag, hipStream_t s) {
    int rc = wall_stress_t<T>(c, u, v, w, z0, log_z0, tau, stats, s, false);
    if (rc) return rc;
    rc = apply_t<T>(c, cfg, tau, ustar, gradp, dt, div, drag, s, nullptr, false);
    if (rc) return rc;
    if (stats || drag) {
        const long nws = band_blocks(c);
        const long nap = apply_tiles(c, cfg);
        hipLaunchKernelGGL(k_finalize_stage, dim3(2), dim3(256), 0, s,
                           (const double*)c->ws_partials, nws, stats,
                           (const double*)c->ap_partials, nap,
                           c->g.dx * c->g.dy * c->g.dz, drag);
        IBM_HIP(hipGetLastError());
    }
    return IBM_OK;
}

}  // namespace

long apply_tiles(const ibm_ctx* c, const TileCfg& cfg) {
    const long nxs = (c->g.nx + 64 * cfg.vx - 1) / (64 * cfg.vx);
    const long njt = (c->g.ny + cfg.ty - 1) / cfg.ty;
    const long nkc = (c->g.nz + cfg.kz - 1) / cfg.kz;
    return nxs * njt * nkc;
}

long band_blocks(const ibm_ctx* c) {
    return std::max<long>(1, (long)nblk(c->rec[0].n, kBandBlock) + (long)nblk(c->rec[1].n, kBandBlock));
}

int size_partials(ibm_ctx* c) {
    // the dense pass may fall back to one element per lane for misaligned
    // views, so size its slots for vx = 1 at the current ty and kz
    TileCfg one = c->cfg;
    one.vx = 1;
    const long need_ap = std::max({3 * std::max(apply_tiles(c, c->cfg), apply_tiles(c, one)),
                                   spectral_slots(c), 3 * sgs_apply_blocks(c)});
    const long need_ws = 4 * band_blocks(c);
    if (need_ap <= c->ap_cap && need_ws <= c->ws_cap) return IBM_OK;
    IBM_HIP(hipDeviceSynchronize());
    if (need_ap > c->ap_cap) {
        (void)hipFree(c->ap_partials);
        c->ap_partials = nullptr;
        c->ap_cap = 0;
        IBM_HIP(hipMalloc(&c->ap_partials, sizeof(double) * (size_t)need_ap));
        c->ap_cap = need_ap;
    }
    if (need_ws > c->ws_cap) {
        (void)hipFree(c->ws_partials);
        c->ws_partials = nullptr;
        c->ws_cap = 0;
        IBM_HIP(hipMalloc(&c->ws_partials, sizeof(double) * (size_t)need_ws));
        c->ws_cap = need_ws;
    }
    return IBM_OK;
}

bool tile_supported(const ibm_ctx* c, const TileCfg& cfg) {
    const int ts = c->dtype == IBM_F64 ? 8 : 4;
    if (cfg.vx != 1 && cfg.vx != 2 && cfg.vx != 4) return false;
    if (cfg.vx * ts > 16) return false;
    if (c->g.nx % cfg.vx) return false;
    if (cfg.ty != 1 && cfg.ty != 2 && cfg.ty != 4 && cfg.ty != 8) return false;
    if (cfg.kz < 1 || cfg.wpb < 1 || cfg.wpb > 4) return false;
    return true;
}

TileCfg default_tile(const ibm_ctx* c) {
    TileCfg t;
    const int ts = c->dtype == IBM_F64 ? 8 : 4;
    const int nx = c->g.nx;
    t.vx = 1;
    for (int vx = 16 / ts; vx >= 2; vx /= 2)
        if (nx % vx == 0 && nx >= 64 * vx) {
            t.vx = vx;
            break;
        }
    // Enough wave-tiles to fill the GPU (1024 SIMDs) with the longest z march
    // that allows: a short march re-reads its halo planes, too few waves leave
    // SIMDs idle.  Float takes one row per wave; double two while that still
    // leaves 1024 waves (rows j-1 and j+1 are then shared by the wave's rows),
    // at most two so the tile stays batchable; four waves per block below 2048
    // waves.  Fitted to tuned tiles of the 512x256x256 hill, the 256x128x128
    // ridge (float and double) and a 128x64x64 hill (double); ibm_autotune
    // times the candidates for a grid.
    constexpr long kFill = 1024;
    t.ty = 1;
    t.kz = 64;
    t.wpb = 1;
    if (ts == 8) {
        t.ty = 2;
        if (apply_tiles(c, t) < kFill) t.ty = 1;
    }
    while (t.kz > 1 && apply_tiles(c, t) < kFill) t.kz /= 2;
    if (apply_tiles(c, t) < 2 * kFill) t.wpb = 4;
    return t;
}

int launch_wall_stress(ibm_ctx* c, const void* u, const void* v, const void* w, double z0,
                       const void* log_z0, void* const tau[6], double* stats, hipStream_t s) {
    if (c->dtype == IBM_F64)
        return wall_stress_t<double>(c, (const double*)u, (const double*)v, (const double*)w, z0,
                                     (const double*)log_z0, tau, stats, s);
    return wall_stress_t<float>(c, (const float*)u, (const float*)v, (const float*)w, z0,
                                (const float*)log_z0, tau, stats, s);
}

int launch_stage(ibm_ctx* c, const TileCfg& cfg, const void* u, const void* v, const void* w,
                 double z0, const void* log_z0, void* const tau[6], void* const ustar[3],
                 const void* const gradp[3], double dt, void* const div[3], double* stats,
                 double* drag, hipStream_t s) {
    if (c->dtype == IBM_F64)
        return stage_t<double>(c, cfg, (const double*)u, (const double*)v, (const double*)w, z0,
                               (const double*)log_z0, tau, ustar, gradp, dt, div, stats, drag, s);
    return stage_t<float>(c, cfg, (const float*)u, (const float*)v, (const float*)w, z0,
                          (const float*)log_z0, tau, ustar, gradp, dt, div, stats, drag, s);
}

int launch_apply(ibm_ctx* c, const TileCfg& cfg, const void* const tau[6], void* const ustar[3],
                 const void* const gradp[3], double dt, void* const div[3], double* drag,
                 hipStream_t s, double* partials) {
    if (c->dtype == IBM_F64)
        return apply_t<double>(c, cfg, tau, ustar, gradp, dt, div, drag, s, partials);
    return apply_t<float>(c, cfg, tau, ustar, gradp, dt, div, drag, s, partials);
}

}  // namespace ibm
