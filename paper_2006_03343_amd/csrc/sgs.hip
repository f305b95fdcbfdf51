// sgs.hip -- the Smagorinsky sub-grid stress with Mason's wall damping (§2.2,
// eqs. t-ij-1963, nu-t, smag, smag-1), the wall distance being the level set
// phi of the node's own grid: the stress field the wall-modeled stage then
// overwrites at band nodes and differentiates.
//
//   S = (grad u + grad u^T) / 2 with the §2.4 differences: central in x and y
//       (periodic), eq. dwdz for dw/dz on uv nodes, eq. dudz for du/dz and
//       dv/dz on w nodes; velocity outside 0 <= k < nz taken as 0;
//   S11, S22, S33, S12 live on uv nodes, S13, S23 on w nodes; |S| =
//       sqrt(2 S:S) on each node set with the other set's components averaged
//       from its nodes above and below;
//   1/lambda^2 = 1/lambda_0^2 + 1/[kappa (phi + z0)]^2, lambda_0 = cs l,
//       l = (dx dy dz)^(1/3), lambda = 0 where phi + z0 <= 0;
//   tau = -2 lambda^2 |S| S.
//
// One wave owns 64 * VX nodes of one row and marches up kz planes.  Per plane
// it loads rows j-1, j, j+1 of u and v (plane k) and of w (plane k+1), the
// centre rows of u and v at k+1 and phi of both grids at k -- every load
// first, then the arithmetic -- and carries the uv-node strain of plane k-1,
// the w-node strain of plane k and w at plane k in registers.  x neighbours
// come from the adjacent lanes (kernels.h: xdiff), y neighbours from the
// loaded rows.  HBM bound: 5 reads (6 with a log z0 field) and 6 writes per
// node; no matrix cores.
#include <algorithm>
#include <cmath>

#include "kernels.h"

// Every product and sum rounded as written: no multiply-add fusion, so the
// result of a node does not depend on the vector width or tile shape that
// computed it.
#pragma clang fp contract(off)

namespace ibm {
namespace {

template <typename T>
struct SgsArgs {
    const T *u, *v, *w, *phi_uv, *phi_w, *log_z0;
    T* tau[6];
    int nx, ny, nz, plane;
    T cx, cy, cz;            // 1/(2 dx), 1/(2 dy), 1/dz
    T inv_l0sq;              // 1 / lambda_0^2
    T kappa, z0;
    int nxs, kz;
    long ntiles;
    int nblocks, per_xcd;
};

// Rows j-1, j, j+1 of one plane of a field and, for lanes 0 and 1, the value
// left and right of the tile in row j (see xdiff).
template <typename T, int VX>
struct Rows {
    Vec<T, VX> m, c, p;
    T e;
};

template <typename T, int VX>
__device__ inline Rows<T, VX> load_rows(const T* __restrict__ f, int pk, int rm, int r0, int rp,
                                        int xlc, int eoff, bool whole_row) {
    Rows<T, VX> r;
    r.m = vload<T, VX>(f + pk + rm + xlc);
    r.c = vload<T, VX>(f + pk + r0 + xlc);
    r.p = vload<T, VX>(f + pk + rp + xlc);
    r.e = whole_row ? T(0) : f[pk + r0 + eoff];
    return r;
}

template <typename T, int VX>
__device__ inline Rows<T, VX> zero_rows() {
    Rows<T, VX> r;
    r.m = r.c = r.p = vzero<T, VX>();
    r.e = T(0);
    return r;
}

// lambda^2 of eq. smag-1 (n = 2): 1 / (1/lambda_0^2 + 1/w^2) written as
// w^2 / (w^2/lambda_0^2 + 1), one quotient, with w = kappa (phi + z0)
template <typename T>
__device__ inline T mixing_sq(const SgsArgs<T>& a, T d, T z0) {
    const T s = d + z0;
    if (!(s > T(0))) return T(0);
    const T wl = a.kappa * s;
    const T w2 = wl * wl;
    return quot_fast(w2, a.inv_l0sq * w2 + T(1));
}

template <typename T, int VX>
__device__ inline void sgs_tile(const SgsArgs<T>& a, long tile, int lane) {
    const int xs = (int)(tile % a.nxs);
    const int t2 = (int)(tile / a.nxs);
    const int j = t2 % a.ny;
    const int kb = (t2 / a.ny) * a.kz;
    const int ke = min(kb + a.kz, a.nz);
    const int nx = a.nx, ny = a.ny, nz = a.nz, plane = a.plane;
    const int x0 = xs * 64 * VX;
    const int xl = x0 + lane * VX;
    const bool act = xl < nx;
    const int xlc = act ? xl : nx - VX;
    const int seg_end = min(nx, x0 + 64 * VX);
    const bool last = act && (xl + VX == seg_end);
    const int xleft = (x0 == 0) ? nx - 1 : x0 - 1;
    const int xright = (seg_end == nx) ? 0 : seg_end;
    const int eoff = (lane & 1) ? xright : xleft;
    const bool whole_row = (x0 == 0) && (seg_end == nx);
    const int last_lane = (seg_end - x0) / VX - 1;
    const int rm = ((j == 0) ? ny - 1 : j - 1) * nx;
    const int r0 = j * nx;
    const int rp = ((j + 1 == ny) ? 0 : j + 1) * nx;
    const T half = T(0.5);

    // uv-node strain of a plane from rows of u and v there and w below/above
    auto uv_strain = [&](const Rows<T, VX>& U, const Rows<T, VX>& V, const Vec<T, VX>& wlo,
                         const Vec<T, VX>& whi, Vec<T, VX> s[4]) {
        const Vec<T, VX> dxu = xdiff<T, VX>(U.c, U.e, lane, last, whole_row, last_lane);
        const Vec<T, VX> dxv = xdiff<T, VX>(V.c, V.e, lane, last, whole_row, last_lane);
#pragma unroll
        for (int e = 0; e < VX; ++e) {
            s[0].v[e] = dxu.v[e] * a.cx;
            s[1].v[e] = (V.p.v[e] - V.m.v[e]) * a.cy;
            s[2].v[e] = (whi.v[e] - wlo.v[e]) * a.cz;
            s[3].v[e] = half * ((U.p.v[e] - U.m.v[e]) * a.cy + dxv.v[e] * a.cx);
        }
    };
    // w-node strain of a plane from u, v at the uv planes above and below it
    // and rows of w there
    auto w_strain = [&](const Vec<T, VX>& uhi, const Vec<T, VX>& ulo, const Vec<T, VX>& vhi,
                        const Vec<T, VX>& vlo, const Rows<T, VX>& W, Vec<T, VX> s[2]) {
        const Vec<T, VX> dxw = xdiff<T, VX>(W.c, W.e, lane, last, whole_row, last_lane);
#pragma unroll
        for (int e = 0; e < VX; ++e) {
            s[0].v[e] = half * ((uhi.v[e] - ulo.v[e]) * a.cz + dxw.v[e] * a.cx);
            s[1].v[e] = half * ((vhi.v[e] - vlo.v[e]) * a.cz + (W.p.v[e] - W.m.v[e]) * a.cy);
        }
    };

    // state at the start of plane kb: uv strain of kb-1, w strain of kb, w at kb
    Vec<T, VX> P[4], Wst[2], wc;
    {
        const bool below = kb > 0;
        const int pb = (kb - 1) * plane, p0 = kb * plane;
        const Rows<T, VX> Ub = below ? load_rows<T, VX>(a.u, pb, rm, r0, rp, xlc, eoff, whole_row)
                                     : zero_rows<T, VX>();
        const Rows<T, VX> Vb = below ? load_rows<T, VX>(a.v, pb, rm, r0, rp, xlc, eoff, whole_row)
                                     : zero_rows<T, VX>();
        const Vec<T, VX> wb = below ? vload<T, VX>(a.w + pb + r0 + xlc) : vzero<T, VX>();
        const Rows<T, VX> Wk = load_rows<T, VX>(a.w, p0, rm, r0, rp, xlc, eoff, whole_row);
        const Vec<T, VX> uk = vload<T, VX>(a.u + p0 + r0 + xlc);
        const Vec<T, VX> vk = vload<T, VX>(a.v + p0 + r0 + xlc);
        if (below) {
            uv_strain(Ub, Vb, wb, Wk.c, P);
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) P[c] = vzero<T, VX>();
        }
        w_strain(uk, Ub.c, vk, Vb.c, Wk, Wst);
        wc = Wk.c;
    }
    for (int k = kb; k < ke; ++k) {
        const int pk = k * plane;
        const bool up = k + 1 < nz;
        // ---- every load of the plane
        const Rows<T, VX> U = load_rows<T, VX>(a.u, pk, rm, r0, rp, xlc, eoff, whole_row);
        const Rows<T, VX> V = load_rows<T, VX>(a.v, pk, rm, r0, rp, xlc, eoff, whole_row);
        Rows<T, VX> Wn;
        Vec<T, VX> un, vn;
        if (up) {
            Wn = load_rows<T, VX>(a.w, pk + plane, rm, r0, rp, xlc, eoff, whole_row);
            un = vload<T, VX>(a.u + pk + plane + r0 + xlc);
            vn = vload<T, VX>(a.v + pk + plane + r0 + xlc);
        } else {
            Wn = zero_rows<T, VX>();
            un = vn = vzero<T, VX>();
        }
        const Vec<T, VX> pu = vload<T, VX>(a.phi_uv + pk + r0 + xlc);
        const Vec<T, VX> pw = vload<T, VX>(a.phi_w + pk + r0 + xlc);
        Vec<T, VX> lz;
        if (a.log_z0) lz = vload<T, VX>(a.log_z0 + pk + r0 + xlc);
        else lz = vzero<T, VX>();
        // ---- strain: uv nodes of plane k, w nodes of plane k+1
        Vec<T, VX> S[4], N[2];
        uv_strain(U, V, wc, Wn.c, S);
        if (up) {
            w_strain(un, U.c, vn, V.c, Wn, N);
        } else {
            N[0] = N[1] = vzero<T, VX>();
        }
        // ---- stress
        Vec<T, VX> t[6];
#pragma unroll
        for (int e = 0; e < VX; ++e) {
            const T z0 = a.log_z0 ? T(exp((double)lz.v[e])) : a.z0;
            // uv node k: S13, S23 from the w nodes k and k+1
            const T s13 = half * (Wst[0].v[e] + N[0].v[e]);
            const T s23 = half * (Wst[1].v[e] + N[1].v[e]);
            const T ss = S[0].v[e] * S[0].v[e] + S[1].v[e] * S[1].v[e] + S[2].v[e] * S[2].v[e] +
                         T(2) * (S[3].v[e] * S[3].v[e] + s13 * s13 + s23 * s23);
            const T nu = mixing_sq(a, pu.v[e], z0) * sqrt_fast(T(2) * ss);
#pragma unroll
            for (int c = 0; c < 4; ++c) t[c].v[e] = T(-2) * nu * S[c].v[e];
            // w node k: S11, S22, S33, S12 from the uv nodes k-1 and k
            T m[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) m[c] = half * (P[c].v[e] + S[c].v[e]);
            const T sw = m[0] * m[0] + m[1] * m[1] + m[2] * m[2] +
                         T(2) * (m[3] * m[3] + Wst[0].v[e] * Wst[0].v[e] + Wst[1].v[e] * Wst[1].v[e]);
            const T nuw = mixing_sq(a, pw.v[e], z0) * sqrt_fast(T(2) * sw);
            t[4].v[e] = T(-2) * nuw * Wst[0].v[e];
            t[5].v[e] = T(-2) * nuw * Wst[1].v[e];
        }
        if (act) {
            const int o = pk + r0 + xl;
#pragma unroll
            for (int c = 0; c < 6; ++c) vstore_nt<T, VX>(a.tau[c] + o, t[c]);
        }
        // ---- carry upward
#pragma unroll
        for (int c = 0; c < 4; ++c) P[c] = S[c];
        Wst[0] = N[0];
        Wst[1] = N[1];
        wc = Wn.c;
    }
}

// XCD-aware: block b runs on XCD b % 8 and takes logical block
// (b % 8) * per_xcd + b / 8, so consecutive tiles share an L2.
template <typename T, int VX>
__global__ void __launch_bounds__(256) k_sgs(SgsArgs<T> a) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpb = blockDim.x >> 6;
    const int lb = (blockIdx.x & 7) * a.per_xcd + (blockIdx.x >> 3);
    const long tile = (long)lb * wpb + wv;
    if (lb < a.nblocks && tile < a.ntiles) sgs_tile<T, VX>(a, tile, lane);
}

template <typename T>
int sgs_t(ibm_ctx* c, const TileCfg& cfg, const T* phi_uv, const T* phi_w, const T* u,
          const T* v, const T* w, double z0, const T* log_z0, double cs, double kappa,
          void* const tau[6], hipStream_t s) {
    SgsArgs<T> a;
    a.u = u;
    a.v = v;
    a.w = w;
    a.phi_uv = phi_uv;
    a.phi_w = phi_w;
    a.log_z0 = log_z0;
    for (int i = 0; i < 6; ++i) a.tau[i] = (T*)tau[i];
    a.nx = c->g.nx;
    a.ny = c->g.ny;
    a.nz = c->g.nz;
    a.plane = c->g.nx * c->g.ny;
    a.cx = (T)(1.0 / (2.0 * c->g.dx));
    a.cy = (T)(1.0 / (2.0 * c->g.dy));
    a.cz = (T)(1.0 / c->g.dz);
    const double l0 = cs * std::cbrt(c->g.dx * c->g.dy * c->g.dz);
    a.inv_l0sq = (T)(1.0 / (l0 * l0));
    a.kappa = (T)kappa;
    a.z0 = (T)z0;
    a.nxs = (c->g.nx + 64 * cfg.vx - 1) / (64 * cfg.vx);
    a.kz = cfg.kz;
    const long nkc = (c->g.nz + cfg.kz - 1) / cfg.kz;
    a.ntiles = (long)a.nxs * c->g.ny * nkc;
    a.nblocks = (int)((a.ntiles + cfg.wpb - 1) / cfg.wpb);
    a.per_xcd = (a.nblocks + 7) / 8;
    const dim3 grid((unsigned)(8 * a.per_xcd)), block((unsigned)(64 * cfg.wpb));
    switch (cfg.vx) {
        case 1: hipLaunchKernelGGL((k_sgs<T, 1>), grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_sgs<T, 2>), grid, block, 0, s, a); break;
        case 4:
            if constexpr (sizeof(T) == 4) {
                hipLaunchKernelGGL((k_sgs<T, 4>), grid, block, 0, s, a);
                break;
            }
            return fail(IBM_E_ARG, "sgs_stress: vx=4 needs float storage");
        default: return fail(IBM_E_ARG, "sgs_stress: unsupported vx=%d", cfg.vx);
    }
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

}  // namespace

int launch_sgs(ibm_ctx* c, const TileCfg& cfg, const void* phi_uv, const void* phi_w,
               const void* u, const void* v, const void* w, double z0, const void* log_z0,
               double cs, double kappa, void* const tau[6], hipStream_t s) {
    if (c->dtype == IBM_F64)
        return sgs_t<double>(c, cfg, (const double*)phi_uv, (const double*)phi_w,
                             (const double*)u, (const double*)v, (const double*)w, z0,
                             (const double*)log_z0, cs, kappa, tau, s);
    return sgs_t<float>(c, cfg, (const float*)phi_uv, (const float*)phi_w, (const float*)u,
                        (const float*)v, (const float*)w, z0, (const float*)log_z0, cs, kappa, tau,
                        s);
}

}  // namespace ibm
