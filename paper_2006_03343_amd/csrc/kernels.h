// kernels.h -- device code of the stage, shared by the per-case kernels
// (stage.hip) and the batched kernels (batch.hip), so that a case computed in
// a batch runs exactly the arithmetic of a plain call.
//
// Wall stress (§3.3): one thread per band record.  It gathers u, v on the uv
// grid and w on the w grid at the record's sample point (trilinear, 24 values
// in 12 x pairs that mostly hit L2), takes the tangential part U_r = u - (u.n)
// n, and writes tau = -c |U_r| (U_r n^T + n U_r^T) with c = (kappa / ln(phi_c /
// z0))^2.  That is the rotation tau_ij = a_im a_jn tau'_mn of the local tensor
// whose only non-zero entries are tau'_13 = tau'_31 = tau_w = -c |U_r|^2 (eq.
// bc-bottom-immersed), written without forming the frame.  uv records store xx,
// yy, zz, xy and w records xz, yz (§3.3).  Other blocks zero the stress of the
// solid nodes of one kSeg-node segment each (§3.3: stress inside the body set
// to zero): a whole block per segment, its mask bytes read first.
//
// Dense pass: one read of the six stress fields and one write of the three
// divergence components per node (HBM bound, no matrix cores).  A wave owns a
// tile of 64*VX nodes along x, TY rows and up to kz planes and marches upward
// in z:
//   * x neighbours come from the adjacent lanes (cross-lane shuffles); the two
//     values beyond the tile ends are loaded with the plane (periodic wrap),
//     or wrap inside the wave when it holds the whole row;
//   * y neighbours: rows j0-1 .. j0+TY of tau_xy, tau_yy and the two halo rows
//     of tau_yz are loaded with the plane;
//   * z neighbours stay in registers from one plane to the next: tau_zz of the
//     plane below and tau_xz, tau_yz of the plane above (loaded one plane
//     ahead);
//   * per plane every load is issued first, branch-free, so a wave waits for
//     memory once per plane; no LDS and no barriers.
// Forcing (eq. u-*-IBM) runs on the kSeg-node segments that hold nodes with
// phi <= 0; the tiles read the 2-bit forcing flags only to leave forced nodes
// out of the drag.  Each
// tile leaves its drag partial in a fixed slot; finalize_slots adds the slots
// in slot order, so results are deterministic and no atomics are used.
#pragma once

#include <cmath>

#include "device.h"
#include "ibm_impl.h"

namespace ibm {

// ----------------------------------------------------------------- wall stress
template <typename T>
struct WSArgs {
    RecView<T> rec[2];
    const T *u, *v, *w, *log_z0;
    T* tau[6];
    const Seg* zsegs;              // segments holding solid nodes
    const uint8_t* mask;           // node classes, one byte per linear index
    int nx, ny, nz;
    long plane;
    int nb_uv, nb_band;            // blocks of uv records, of all records (>= 1)
    double ln_scalar;              // ln(phi_c / z0) for a scalar z0
    double ln_phic;                // ln(phi_c) for a per-node log z0
    double kappa;
    double dz;
    double* partials;              // 4 per band block
    double* stats;                 // nullable
};

template <typename T>
__device__ inline T trilerp(const T* __restrict__ f, long c00, long c10, long c01, long c11,
                            long z0, long z1, T fx, T fy, T fz) {
    const T gx = T(1) - fx, gy = T(1) - fy, gz = T(1) - fz;
    T a0 = f[z0 + c00] * gx + f[z0 + c10] * fx;
    T b0 = f[z0 + c01] * gx + f[z0 + c11] * fx;
    T a1 = f[z1 + c00] * gx + f[z1 + c10] * fx;
    T b1 = f[z1 + c01] * gx + f[z1 + c11] * fx;
    T lo = a0 * gy + b0 * fy;
    T hi = a1 * gy + b1 * fy;
    return lo * gz + hi * fz;
}

// The x-neighbour pair f[off], f[off + sx] of a sample stencil: one 8-byte
// (16-byte for double) load where the pair is contiguous (sx = 1), two loads
// across the periodic seam.  Global loads of several dwords need only 4-byte
// alignment.
template <typename T>
__device__ inline void load_xpair(const T* __restrict__ f, long off, long sx, T& lo, T& hi) {
    if (sx == 1) {
        typedef T T2 __attribute__((ext_vector_type(2))) __attribute__((aligned(sizeof(T))));
        const T2 p = *reinterpret_cast<const T2*>(f + off);
        lo = p.x;
        hi = p.y;
    } else {
        lo = f[off];
        hi = f[off + sx];
    }
}

// trilerp with the four x pairs loaded by load_xpair (c10 = c00 + sx,
// c11 = c01 + sx); the same arithmetic in the same order.
template <typename T>
__device__ inline T trilerp_xpair(const T* __restrict__ f, long c00, long c01, long sx, long z0,
                                  long z1, T fx, T fy, T fz) {
    const T gx = T(1) - fx, gy = T(1) - fy, gz = T(1) - fz;
    T p00, p10, p01, p11, q00, q10, q01, q11;
    load_xpair<T>(f, z0 + c00, sx, p00, p10);
    load_xpair<T>(f, z0 + c01, sx, p01, p11);
    load_xpair<T>(f, z1 + c00, sx, q00, q10);
    load_xpair<T>(f, z1 + c01, sx, q01, q11);
    T a0 = p00 * gx + p10 * fx;
    T b0 = p01 * gx + p11 * fx;
    T a1 = q00 * gx + q10 * fx;
    T b1 = q01 * gx + q11 * fx;
    T lo = a0 * gy + b0 * fy;
    T hi = a1 * gy + b1 * fy;
    return lo * gz + hi * fz;
}

// Stress of the solid nodes of one segment set to zero (class code 2, or 3:
// the body interior of Chester et al.'s classes), by ``nthr`` threads
// numbered ``tid``: thread tid takes nodes q + tid + i * nthr, so each store
// of a wave is contiguous.  kPer mask bytes per thread are loaded before any
// store (byte loads may alias the stores, so the compiler would not hoist
// them); offsets are 32-bit (a context holds fewer than 2^31 nodes).
template <typename T>
__device__ inline void zero_seg(const WSArgs<T>& a, const Seg sg, int tid, int nthr) {
    constexpr int kPer = 4;
    const uint8_t* __restrict__ mk = a.mask + sg.q;
    T* __restrict__ t0 = a.tau[0] + sg.q;
    T* __restrict__ t1 = a.tau[1] + sg.q;
    T* __restrict__ t2 = a.tau[2] + sg.q;
    T* __restrict__ t3 = a.tau[3] + sg.q;
    T* __restrict__ t4 = a.tau[4] + sg.q;
    T* __restrict__ t5 = a.tau[5] + sg.q;
    for (int o = tid; o < sg.len; o += kPer * nthr) {
        uint32_t m[kPer];
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int t = o + i * nthr;
            m[i] = t < sg.len ? mk[t] : 0u;
        }
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int t = o + i * nthr;
            if ((m[i] & 3u) >= 2u) {
                t0[t] = T(0);
                t1[t] = T(0);
                t2[t] = T(0);
                t3[t] = T(0);
            }
            if (((m[i] >> 2) & 3u) >= 2u) {
                t4[t] = T(0);
                t5[t] = T(0);
            }
        }
    }
}

// One block of the wall-stress pass: block b < nb_band handles kBandBlock band
// records (uv records first, then w records) and leaves its statistics in slot
// b; block b >= nb_band zeroes the solid nodes of segment b - nb_band.
template <typename T, bool MIXED, bool HAS_LZ>
__device__ inline void ws_block(const WSArgs<T>& a, int b) {
    if (b >= a.nb_band) {
        zero_seg<T>(a, a.zsegs[b - a.nb_band], threadIdx.x, blockDim.x);
        return;
    }
    const int kind = b < a.nb_uv ? IBM_GRID_UV : IBM_GRID_W;
    const RecView<T>& R = a.rec[kind];
    const long r = (long)(kind == IBM_GRID_UV ? b : b - a.nb_uv) * kBandBlock + threadIdx.x;
    double tw_acc = 0.0, umax = 0.0, cnt = 0.0;
    if (r < R.n) {
        const long q = R.q[r];
        const T n0 = R.nx[r], n1 = R.ny[r], n2 = R.nz[r];
        const long c00 = R.base[r], sx = R.sx[r], c01 = c00 + R.sy[r];
        const T fx = R.fx[r], fy = R.fy[r];
        const int ku = R.ku[r], kw = R.kw[r];
        const long zu0 = ku * a.plane, zu1 = min(ku + 1, a.nz - 1) * a.plane;
        const long zw0 = kw * a.plane, zw1 = min(kw + 1, a.nz - 1) * a.plane;
        const T fzu = R.fzu[r], fzw = R.fzw[r];
        const T us = trilerp_xpair<T>(a.u, c00, c01, sx, zu0, zu1, fx, fy, fzu);
        const T vs = trilerp_xpair<T>(a.v, c00, c01, sx, zu0, zu1, fx, fy, fzu);
        const T ws = trilerp_xpair<T>(a.w, c00, c01, sx, zw0, zw1, fx, fy, fzw);
        const T un = us * n0 + vs * n1 + ws * n2;
        const T ur0 = us - un * n0, ur1 = vs - un * n1, ur2 = ws - un * n2;
        const T U = sqrt(ur0 * ur0 + ur1 * ur1 + ur2 * ur2);
        // c |U_r|, with c = (kappa / ln(phi_c / z0))^2
        T cU;
        if (MIXED && fabs((double)R.phi[r]) <= a.dz) {
            const double lnr = HAS_LZ ? a.ln_phic - (double)a.log_z0[q] : a.ln_scalar;
            const double k_l = a.kappa / lnr;
            cU = (T)(k_l * k_l * (double)U);
        } else {
            const T lnr = HAS_LZ ? T(a.ln_phic) - a.log_z0[q] : T(a.ln_scalar);
            const T k_l = T(a.kappa) / lnr;
            cU = k_l * k_l * U;
        }
        if (kind == IBM_GRID_UV) {
            a.tau[0][q] = -cU * (T(2) * ur0 * n0);
            a.tau[1][q] = -cU * (T(2) * ur1 * n1);
            a.tau[2][q] = -cU * (T(2) * ur2 * n2);
            a.tau[3][q] = -cU * (ur0 * n1 + n0 * ur1);
        } else {
            a.tau[4][q] = -cU * (ur0 * n2 + n0 * ur2);
            a.tau[5][q] = -cU * (ur1 * n2 + n1 * ur2);
        }
        tw_acc = -(double)cU * (double)U;
        umax = (double)U;
        cnt = 1.0;
    }
    if (!a.stats) return;
    // block partial: [sum tau_w uv, sum tau_w w, max |U_r|, count]; k_finalize adds the
    // slots in slot order after the kernel
    __shared__ double red[3][kBandBlock / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double s = wave_sum(tw_acc), m = wave_max(umax), c = wave_sum(cnt);
    if (lane == 0) {
        red[0][wv] = s;
        red[1][wv] = m;
        red[2][wv] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ss = 0.0, mm = 0.0, cc = 0.0;
        for (int i = 0; i < kBandBlock / 64; ++i) {
            ss += red[0][i];
            mm = fmax(mm, red[1][i]);
            cc += red[2][i];
        }
        double* p = a.partials + 4 * (long)b;
        p[0] = kind == IBM_GRID_UV ? ss : 0.0;
        p[1] = kind == IBM_GRID_W ? ss : 0.0;
        p[2] = mm;
        p[3] = cc;
    }
}

// Fixed-order reduction of per-slot partials (one block): out[c] = scale_c *
// (sum or max over slots i of p[i * nc + c]); bit ``c`` of maxmask selects max.
__device__ inline void finalize_slots(const double* __restrict__ p, long nslots, int nc,
                                      unsigned maxmask, double scale, double* __restrict__ out) {
    // thread t takes slots t, t + B, t + 2B, ... (B = blockDim.x), four per
    // step with their loads issued together; then a fixed-order wave and block
    // combine: deterministic for a given block size
    constexpr int kU = 4;
    __shared__ double red[4][16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const long B = blockDim.x;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    auto add = [&](int c, double x) {
        acc[c] = ((maxmask >> c) & 1u) ? fmax(acc[c], x) : acc[c] + x;
    };
    long i = threadIdx.x;
    for (; i + (kU - 1) * B < nslots; i += kU * B) {
        double x[kU][4];
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
            for (int c = 0; c < 4; ++c) x[u][c] = c < nc ? p[(i + u * B) * nc + c] : 0.0;
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < nc) add(c, x[u][c]);
    }
    for (; i < nslots; i += B)
        for (int c = 0; c < nc; ++c) add(c, p[i * nc + c]);
    for (int c = 0; c < nc; ++c) {
        const double r = ((maxmask >> c) & 1u) ? wave_max(acc[c]) : wave_sum(acc[c]);
        if (lane == 0) red[c][wv] = r;
    }
    __syncthreads();
    if (threadIdx.x < nc) {
        const int c = threadIdx.x;
        const bool mx = (maxmask >> c) & 1u;
        double r = red[c][0];
        for (int w = 1; w < nw; ++w) r = mx ? fmax(r, red[c][w]) : r + red[c][w];
        out[c] = mx ? r : scale * r;
    }
    __syncthreads();
}

// One fixed-order reduction: nslots slots of nc doubles into out[nc].
struct FinJob {
    const double* p;
    long nslots;
    int nc;
    unsigned maxmask;   // bit c: component c is a maximum, not a sum
    double scale;       // applied to the sums
    double* out;
};

// ----------------------------------------------------------------- dense pass
template <typename T>
struct ApplyArgs {
    const T* tau[6];
    T* ustar[3];
    const T* gradp[3];
    T* div[3];
    const uint32_t* fmask;
    const uint8_t* mask;     // node classes and forcing flags, one byte per node
    int nx, ny, nz, wrow;
    long plane;
    T cx, cy, cz;            // 1/(2 dx), 1/(2 dy), 1/dz
    T fdt;                   // 3 dt / 2
    int nxs, njt, kz;        // x segments, row tiles, planes per tile
    long ntiles;
    int nblocks;             // blocks that own tiles (the grid is padded to a multiple of 8)
    int per_xcd;             // logical blocks per XCD
    double* partials;        // 3 per tile
    double* drag;            // nullable
    const Seg* fsegs;        // segments holding forced nodes
    int nfblocks;            // blocks after the tile blocks that force
    long nfsegs;
    double dv;
};

template <typename T>
__device__ inline T readlane(T x, int l) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
    } else {
        const long long b = __builtin_bit_cast(long long, x);
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
        return __builtin_bit_cast(T, ((long long)hi << 32) | (unsigned)lo);
    }
}

// Central difference along x of a lane-distributed row: (f[x+1] - f[x-1]).
// Neighbours inside the wave come from the adjacent lanes.  When the wave
// holds the whole periodic row the ends wrap inside the wave; otherwise lane
// 0 holds the value left of the segment and lane 1 the value right of it
// (``edge``, loaded with the rest of the plane) and both are broadcast.
template <typename T, int VX>
__device__ inline Vec<T, VX> xdiff(const Vec<T, VX>& r, T edge, int lane, bool last,
                                   bool whole_row, int last_lane) {
    T lft = __shfl_up(r.v[VX - 1], 1, 64);
    T rgt = __shfl_down(r.v[0], 1, 64);
    T hl, hr;
    if (whole_row) {
        hl = readlane(r.v[VX - 1], last_lane);
        hr = readlane(r.v[0], 0);
    } else {
        hl = readlane(edge, 0);
        hr = readlane(edge, 1);
    }
    if (lane == 0) lft = hl;
    if (last) rgt = hr;
    Vec<T, VX> d;
#pragma unroll
    for (int e = 0; e < VX; ++e) {
        const T hi = (e == VX - 1) ? rgt : r.v[e + 1];
        const T lo = (e == 0) ? lft : r.v[e - 1];
        d.v[e] = hi - lo;
    }
    return d;
}

// The dense pass.  Per plane every load is issued first, without branches
// (lanes past the end of the row read a valid clamped address and discard
// it), so a wave waits for memory once per plane.
// Direct forcing (eq. u-*-IBM) of the forced nodes of one segment, by
// ``nthr`` threads numbered ``tid`` taking nodes q + tid + i * nthr; per round
// of kPer nodes a thread loads the mask bytes, then the pressure gradient of
// its forced nodes (exec-masked loads), then stores, so it waits for memory
// twice per round.
template <typename T>
__device__ inline void force_seg(const ApplyArgs<T>& a, const Seg sg, int tid, int nthr) {
    constexpr int kPer = 4;
    const uint8_t* __restrict__ mk = a.mask + sg.q;
    const T* __restrict__ g0 = a.gradp[0] ? a.gradp[0] + sg.q : nullptr;
    const T* __restrict__ g1 = a.gradp[1] ? a.gradp[1] + sg.q : nullptr;
    const T* __restrict__ g2 = a.gradp[2] ? a.gradp[2] + sg.q : nullptr;
    T* __restrict__ u0 = a.ustar[0] + sg.q;
    T* __restrict__ u1 = a.ustar[1] + sg.q;
    T* __restrict__ u2 = a.ustar[2] + sg.q;
    const T f = a.fdt;
    for (int o = tid; o < sg.len; o += kPer * nthr) {
        uint32_t m[kPer];
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int t = o + i * nthr;
            m[i] = t < sg.len ? mk[t] : 0u;
        }
        T p0[kPer], p1[kPer], p2[kPer];
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int t = o + i * nthr;
            p0[i] = p1[i] = p2[i] = T(0);
            if (m[i] & 16u) {
                if (g0) p0[i] = g0[t];
                if (g1) p1[i] = g1[t];
            }
            if ((m[i] & 32u) && g2) p2[i] = g2[t];
        }
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int t = o + i * nthr;
            if (m[i] & 16u) {
                u0[t] = g0 ? f * p0[i] : T(0);
                u1[t] = g1 ? f * p1[i] : T(0);
            }
            if (m[i] & 32u) u2[t] = g2 ? f * p2[i] : T(0);
        }
    }
}

// One wave-tile of the dense pass (see the file comment): divergence of the
// tile's nodes and, if a.drag, the tile's drag partial in slot ``tile``.
// Wave-uniform: every lane of the wave calls it with the same tile.
template <typename T, typename Acc, int VX, int TY>
__device__ inline void apply_tile(const ApplyArgs<T>& a, long tile, int lane) {
    Acc s0 = Acc(0), s1 = Acc(0), s2 = Acc(0);
    const int xs = (int)(tile % a.nxs);
    const int t2 = (int)(tile / a.nxs);
    const int jt = t2 % a.njt;
    const int kb = (t2 / a.njt) * a.kz;
    const int ke = min(kb + a.kz, a.nz);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int plane = (int)a.plane;
    const int x0 = xs * 64 * VX;
    const int xl = x0 + lane * VX;
    const bool act = xl < nx;
    const int xlc = act ? xl : nx - VX;          // always a valid vector address
    const int seg_end = min(nx, x0 + 64 * VX);
    const bool last = act && (xl + VX == seg_end);
    const int xleft = (x0 == 0) ? nx - 1 : x0 - 1;
    const int xright = (seg_end == nx) ? 0 : seg_end;
    const int eoff = (lane & 1) ? xright : xleft; // lane 0: left edge, lane 1: right edge
    const bool whole_row = (x0 == 0) && (seg_end == nx);   // wave-uniform
    const int last_lane = (seg_end - x0) / VX - 1;
    const int j0 = jt * TY;
    int roff[TY + 2];   // offset of row j0-1+r (r = 0..TY+1), periodic in y
    int frow[TY];       // forcing-flag row of tile row r (clamped for ragged tiles)
#pragma unroll
    for (int r = 0; r < TY + 2; ++r) {
        int jj = (j0 - 1 + r) % ny;
        if (jj < 0) jj += ny;
        roff[r] = jj * nx;
    }
#pragma unroll
    for (int r = 0; r < TY; ++r) frow[r] = min(j0 + r, ny - 1);
    const T *txx = a.tau[0], *tyy = a.tau[1], *tzz = a.tau[2], *txy = a.tau[3],
            *txz = a.tau[4], *tyz = a.tau[5];
    Vec<T, VX> zz_prev[TY], xz_cur[TY], yz_cur[TY];
    {
        const int pk = kb * plane;
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            xz_cur[r] = vload<T, VX>(txz + pk + roff[r + 1] + xlc);
            yz_cur[r] = vload<T, VX>(tyz + pk + roff[r + 1] + xlc);
            zz_prev[r] = (kb > 0) ? vload<T, VX>(tzz + pk - plane + roff[r + 1] + xlc)
                                  : vzero<T, VX>();
        }
    }
    const uint32_t mbits = (1u << (2 * VX)) - 1u;
    const int fsh = 2 * (xlc & 15);
    for (int k = kb; k < ke; ++k) {
        const int pk = k * plane;
        const bool has_up = k + 1 < nz;
        // ---- issue every load of plane k
        Vec<T, VX> xy[TY + 2], yy[TY + 2], xx[TY], zz[TY], xzn[TY], yzn[TY];
        T exx[TY], exy[TY], exz[TY];
        uint32_t fw[TY];
#pragma unroll
        for (int r = 0; r < TY + 2; ++r) {
            xy[r] = vload<T, VX>(txy + pk + roff[r] + xlc);
            yy[r] = vload<T, VX>(tyy + pk + roff[r] + xlc);
        }
        const Vec<T, VX> yz_lo = vload<T, VX>(tyz + pk + roff[0] + xlc);
        const Vec<T, VX> yz_hi = vload<T, VX>(tyz + pk + roff[TY + 1] + xlc);
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            const int rb = pk + roff[r + 1];
            xx[r] = vload<T, VX>(txx + rb + xlc);
            zz[r] = vload<T, VX>(tzz + rb + xlc);
            if (has_up) {
                xzn[r] = vload<T, VX>(txz + rb + plane + xlc);
                yzn[r] = vload<T, VX>(tyz + rb + plane + xlc);
            } else {
                xzn[r] = vzero<T, VX>();
                yzn[r] = vzero<T, VX>();
            }
            if (!whole_row) {
                exx[r] = txx[rb + eoff];
                exy[r] = txy[rb + eoff];
                exz[r] = txz[rb + eoff];
            } else {
                exx[r] = exy[r] = exz[r] = T(0);
            }
            fw[r] = a.fmask[(k * ny + frow[r]) * a.wrow + (xlc >> 4)];
        }
        // ---- compute the TY rows
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            const Vec<T, VX> dxx = xdiff<T, VX>(xx[r], exx[r], lane, last, whole_row, last_lane);
            const Vec<T, VX> dxy = xdiff<T, VX>(xy[r + 1], exy[r], lane, last, whole_row, last_lane);
            const Vec<T, VX> dxz = xdiff<T, VX>(xz_cur[r], exz[r], lane, last, whole_row, last_lane);
            const Vec<T, VX>& yz_dn = (r == 0) ? yz_lo : yz_cur[r - 1];
            const Vec<T, VX>& yz_up = (r + 1 == TY) ? yz_hi : yz_cur[r + 1];
            if (act && j0 + r < ny) {
                Vec<T, VX> dvx, dvy, dvz;
#pragma unroll
                for (int e = 0; e < VX; ++e) {
                    dvx.v[e] = dxx.v[e] * a.cx + (xy[r + 2].v[e] - xy[r].v[e]) * a.cy +
                               (xzn[r].v[e] - xz_cur[r].v[e]) * a.cz;
                    dvy.v[e] = dxy.v[e] * a.cx + (yy[r + 2].v[e] - yy[r].v[e]) * a.cy +
                               (yzn[r].v[e] - yz_cur[r].v[e]) * a.cz;
                    dvz.v[e] = dxz.v[e] * a.cx + (yz_up.v[e] - yz_dn.v[e]) * a.cy +
                               (zz[r].v[e] - zz_prev[r].v[e]) * a.cz;
                }
                const int o = pk + roff[r + 1] + xl;
                vstore_nt<T, VX>(a.div[0] + o, dvx);
                vstore_nt<T, VX>(a.div[1] + o, dvy);
                vstore_nt<T, VX>(a.div[2] + o, dvz);
                const uint32_t fb = (fw[r] >> fsh) & mbits;
#pragma unroll
                for (int e = 0; e < VX; ++e) {
                    if (!((fb >> (2 * e)) & 1u)) {
                        s0 += (Acc)dvx.v[e];
                        s1 += (Acc)dvy.v[e];
                    }
                    if (!((fb >> (2 * e + 1)) & 1u)) s2 += (Acc)dvz.v[e];
                }
            }
        }
        // ---- carry the plane upward
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            zz_prev[r] = zz[r];
            xz_cur[r] = xzn[r];
            yz_cur[r] = yzn[r];
        }
    }
    if (!a.drag) return;
    const double d0 = wave_sum((double)s0), d1 = wave_sum((double)s1), d2 = wave_sum((double)s2);
    if (lane == 0) {
        a.partials[3 * tile + 0] = d0;
        a.partials[3 * tile + 1] = d1;
        a.partials[3 * tile + 2] = d2;
    }
}

// ------------------------------------------------------------ host-side set-up
inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename T>
inline WSArgs<T> make_ws_args(const ibm_ctx* c, const T* u, const T* v, const T* w, double z0,
                              const T* log_z0, void* const tau[6], double* stats) {
    WSArgs<T> a;
    a.rec[0] = view<T>(c->rec[0]);
    a.rec[1] = view<T>(c->rec[1]);
    a.u = u;
    a.v = v;
    a.w = w;
    a.log_z0 = log_z0;
    for (int i = 0; i < 6; ++i) a.tau[i] = (T*)tau[i];
    a.zsegs = c->zsegs;
    a.mask = c->mask;
    a.nx = c->g.nx;
    a.ny = c->g.ny;
    a.nz = c->g.nz;
    a.plane = (long)c->g.nx * c->g.ny;
    a.nb_uv = (int)nblk(c->rec[0].n, kBandBlock);
    a.nb_band = (int)band_blocks(c);
    a.ln_scalar = log_z0 ? 0.0 : std::log(c->p.phi_c / z0);
    a.ln_phic = std::log(c->p.phi_c);
    a.kappa = c->p.kappa;
    a.dz = c->g.dz;
    a.partials = c->ws_partials;
    a.stats = stats;
    return a;
}

template <typename T>
inline ApplyArgs<T> make_apply_args(const ibm_ctx* c, const TileCfg& cfg, const void* const tau[6],
                                    void* const ustar[3], const void* const gradp[3], double dt,
                                    void* const div[3], double* drag) {
    ApplyArgs<T> a;
    for (int i = 0; i < 6; ++i) a.tau[i] = (const T*)tau[i];
    for (int i = 0; i < 3; ++i) {
        a.ustar[i] = (T*)ustar[i];
        a.gradp[i] = gradp ? (const T*)gradp[i] : nullptr;
        a.div[i] = (T*)div[i];
    }
    a.fmask = c->fmask;
    a.mask = c->mask;
    a.nx = c->g.nx;
    a.ny = c->g.ny;
    a.nz = c->g.nz;
    a.wrow = c->wrow;
    a.plane = (long)c->g.nx * c->g.ny;
    a.cx = (T)(1.0 / (2.0 * c->g.dx));
    a.cy = (T)(1.0 / (2.0 * c->g.dy));
    a.cz = (T)(1.0 / c->g.dz);
    a.fdt = (T)(1.5 * dt);
    a.nxs = (c->g.nx + 64 * cfg.vx - 1) / (64 * cfg.vx);
    a.njt = (c->g.ny + cfg.ty - 1) / cfg.ty;
    a.kz = cfg.kz;
    const long nkc = (c->g.nz + cfg.kz - 1) / cfg.kz;
    a.ntiles = (long)a.nxs * a.njt * nkc;
    a.nblocks = (int)((a.ntiles + cfg.wpb - 1) / cfg.wpb);
    a.per_xcd = (a.nblocks + 7) / 8;
    a.partials = c->ap_partials;
    a.drag = drag;
    a.dv = c->g.dx * c->g.dy * c->g.dz;
    a.fsegs = c->fsegs;
    a.nfsegs = c->nfsegs;
    a.nfblocks = 0;
    return a;
}

}  // namespace ibm
