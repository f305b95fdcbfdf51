// sgs_apply.hip -- the Smagorinsky stress with Mason's damping (§2.2, as
// ibm_sgs_stress computes it) and the stage's dense pass (§2.4 divergence,
// eq. u-*-IBM forcing, drag; as ibm_apply) in one pass, so the sub-grid stress
// is never written to memory and read back.
//
// The stress the divergence differentiates is, node by node and on each node
// set, the wall-model stress where the node is a band node of its grid (read
// from tau, which ibm_wall_stress has filled there), 0 where it is solid, and
// the Smagorinsky stress of the velocity elsewhere -- the field ibm_sgs_stress
// followed by ibm_wall_stress leaves in tau.
//
// A block of kWaves waves owns kRows rows j0 .. j0+kRows-1 of an x segment
// and a chunk of planes.  Wave wv computes the stress of row j0-1+wv (the
// two outer waves: the y halo) on 64 consecutive nodes, one per lane: the
// segment's 60 and 2 on either side.  The strain, and with it the stress, is
// wrong on the outermost node of each side, which no output needs: x
// differences come from the adjacent lanes without edge loads.  Per plane the
// components differenced in y (tau_xy, tau_yy on uv nodes, tau_yz on w nodes)
// go through LDS (three plane buffers, so one barrier per plane suffices), z
// differences stay in registers.  The uv divergence of plane k needs tau_xz,
// tau_yz on w plane k+1, which the march reaches one plane later, so it is
// formed one plane behind the w divergence; a chunk starts one plane below
// its first (the march state rebuilt from the velocities there) and, unless
// it is the top one, ends one plane above its last.
//
// Loads go through buffer resources based at the block's slab of planes, so
// a wave adds row and plane offsets in scalar registers; in float a plane's
// loads are issued two planes ahead of its arithmetic.  The work is the
// Smagorinsky arithmetic of 8 rows for 6 and 64 nodes for 60: the pass is
// bound by that arithmetic and the barrier per plane, not by HBM.
//
// Bytes per node: u, v, w, phi_uv, phi_w (log z0) in, the class byte, the
// band stress where there is one, div out; the halo rows and columns of a
// block are the interior rows of its neighbours (L2).
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "kernels.h"

// Every product and sum rounded as written, as in the Smagorinsky kernel.
#pragma clang fp contract(off)

namespace ibm {
namespace {

constexpr int kRows = 6;             // divergence rows per block (8 waves: two blocks per CU)
constexpr int kWaves = kRows + 2;    // one stress row per wave: rows j0-1 .. j0+kRows
constexpr int kChunk = 32;           // planes per block (fewer where a slab passes 4 GiB)

template <int VX>
constexpr int halo() { return VX > 2 ? VX : 2; }
template <int VX>
constexpr int span() { return 64 * VX - 2 * halo<VX>(); }   // x nodes per block written

template <typename T>
struct FusedArgs {
    const T *u, *v, *w, *phi_uv, *phi_w, *log_z0;
    int nx, ny, nz, plane;
    T cx, cy, cz;            // 1/(2 dx), 1/(2 dy), 1/dz
    T inv_l0sq;              // 1 / lambda_0^2
    T kappa, z0;
    int nxs, njb;            // x segments, row blocks
    int kc;                  // planes per block
    int nblocks;             // dense blocks (nxs * njb * z chunks)
    int per_xcd;             // logical dense blocks per XCD
    ApplyArgs<T> ap;         // tau (band values), ustar, gradp, div, mask, forcing segments, drag
};

// lambda^2 of eq. smag-1 (n = 2): 1 / (1/lambda_0^2 + 1/w^2) written as
// w^2 / (w^2/lambda_0^2 + 1), one quotient, with w = kappa (phi + z0)
template <typename T>
__device__ inline T mixing_sq(const FusedArgs<T>& a, T d, T z0) {
    const T s = d + z0;
    if (!(s > T(0))) return T(0);
    const T wl = a.kappa * s;
    const T w2 = wl * wl;
    return quot_fast(w2, a.inv_l0sq * w2 + T(1));
}

__device__ inline int wrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// Rows j-1, j, j+1 of one plane of a field at this lane's VX nodes.
template <typename T, int VX>
struct Row3 {
    Vec<T, VX> m, c, p;
};

// The input fields over a block's slab -- its chunk of planes, two planes
// below and one above -- as buffer resources based at the slab's first plane
// kbase: a load takes the lane's byte offset and a uniform byte offset within
// the slab (32-bit; the host keeps a slab under 4 GiB).
struct SlabIn {
    Rsrc u, v, w, pu, pw, lz, mask;
};

// rows rm, r0, rp of the slab plane starting at node pk, at the lane's byte offset xo
template <typename T, int VX>
__device__ inline Row3<T, VX> load3(Rsrc f, unsigned pk, unsigned rm, unsigned r0, unsigned rp,
                                   unsigned xo) {
    constexpr unsigned S = sizeof(T);
    Row3<T, VX> r;
    r.m = bload<T, VX>(f, xo, (pk + rm) * S);
    r.c = bload<T, VX>(f, xo, (pk + r0) * S);
    r.p = bload<T, VX>(f, xo, (pk + rp) * S);
    return r;
}

template <typename T, int VX>
__device__ inline Row3<T, VX> zero3() {
    Row3<T, VX> r;
    r.m = r.c = r.p = vzero<T, VX>();
    return r;
}

// Everything the march reads at one plane k of its row.
template <typename T, int VX>
struct PlaneIn {
    Row3<T, VX> U, V, Wn;          // u, v at k; w at k+1
    Vec<T, VX> un, vn, pu, pw, lz; // u, v at k+1; phi of both grids, ln z0 at k
    uint32_t m[VX];                // class bytes at k
};

template <typename T, int VX>
__device__ inline void load_plane(const FusedArgs<T>& a, const SlabIn& sl, int k, int kbase,
                                  unsigned rm, unsigned r0, unsigned rp, unsigned x,
                                  PlaneIn<T, VX>& in) {
    static_assert(VX == 1, "one node per lane");
    constexpr unsigned S = sizeof(T);
    const unsigned pk = (unsigned)(k - kbase) * (unsigned)a.plane;   // plane k in the slab
    const unsigned pn = pk + (unsigned)a.plane;
    const unsigned xo = x * S;
    const bool up = k + 1 < a.nz;
    in.U = load3<T, VX>(sl.u, pk, rm, r0, rp, xo);
    in.V = load3<T, VX>(sl.v, pk, rm, r0, rp, xo);
    in.Wn = up ? load3<T, VX>(sl.w, pn, rm, r0, rp, xo) : zero3<T, VX>();
    in.un = up ? bload<T, VX>(sl.u, xo, (pn + r0) * S) : vzero<T, VX>();
    in.vn = up ? bload<T, VX>(sl.v, xo, (pn + r0) * S) : vzero<T, VX>();
    in.pu = bload<T, VX>(sl.pu, xo, (pk + r0) * S);
    in.pw = bload<T, VX>(sl.pw, xo, (pk + r0) * S);
    in.lz = a.log_z0 ? bload<T, VX>(sl.lz, xo, (pk + r0) * S) : vzero<T, VX>();
    in.m[0] = bload_u8(sl.mask, x, pk + r0);
}

// PF: how many planes ahead of the march a plane's loads are issued
template <typename T, typename Acc, int VX, int PF>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(4)))
k_sgs_apply(FusedArgs<T> a) {
    static_assert(PF == 1 || PF == 2, "loads one or two planes ahead");
    constexpr int H = halo<VX>(), SPAN = span<VX>();
    const ApplyArgs<T>& ap = a.ap;
    const int dense = 8 * a.per_xcd;
    if ((int)blockIdx.x >= dense) {
        // forcing: quarters of the forcing segments
        constexpr int kPiece = kSeg / 4;
        for (long it = blockIdx.x - dense; it < 4 * ap.nfsegs; it += ap.nfblocks) {
            const Seg sg = ap.fsegs[it >> 2];
            const int off = (int)(it & 3) * kPiece;
            if (off < sg.len)
                force_seg<T>(ap, Seg{sg.q + off, min(kPiece, sg.len - off), 0, 0}, threadIdx.x,
                             blockDim.x);
        }
        return;
    }
    // XCD-aware: block b runs on XCD b % 8 and takes logical block
    // (b % 8) * per_xcd + b / 8, so neighbouring row blocks share an L2
    const int lb = (blockIdx.x & 7) * a.per_xcd + (blockIdx.x >> 3);
    if (lb >= a.nblocks) return;                         // the whole block
    __shared__ T sh[3][3][kWaves][64 * VX];              // [plane % 3][xy, yy, yz][row][node]
    __shared__ double red[3][kWaves];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nx = a.nx, ny = a.ny, nz = a.nz, plane = a.plane;
    const int xs = lb % a.nxs, t2 = lb / a.nxs;
    const int jb = t2 % a.njb, chunk = t2 / a.njb;
    const int kb = chunk * a.kc, ke = min(kb + a.kc, nz);
    const int x0 = xs * SPAN;
    const int jr = jb * kRows - 1 + wv;                  // this wave's row, unwrapped
    const int j = wrap(jr, ny);
    const int xb = x0 - H + VX * lane;                   // this lane's first node, unwrapped
    const unsigned x = wrap(xb, nx);                     // nx % VX == 0: no wrap inside the lane
    const unsigned xo = x * (unsigned)sizeof(T);        // its byte offset in a row (loads)
    const bool row_out = wv >= 1 && wv <= kRows && jr < ny;
    bool outn[VX];
#pragma unroll
    for (int e = 0; e < VX; ++e) outn[e] = row_out && xb + e >= x0 && xb + e < min(x0 + SPAN, nx);
    const int rm = wrap(j - 1, ny) * nx, r0 = j * nx, rp = wrap(j + 1, ny) * nx;
    // the slab: planes kbase .. ke + 1 of every input field
    const int kbase = max(kb - 2, 0);
    const long sb = (long)kbase * plane;
    SlabIn sl;
    sl.u = buffer_rsrc(a.u + sb);
    sl.v = buffer_rsrc(a.v + sb);
    sl.w = buffer_rsrc(a.w + sb);
    sl.pu = buffer_rsrc(a.phi_uv + sb);
    sl.pw = buffer_rsrc(a.phi_w + sb);
    sl.lz = buffer_rsrc(a.log_z0 ? a.log_z0 + sb : a.u + sb);
    sl.mask = buffer_rsrc(ap.mask + sb);
    const bool last = lane == 63;
    const T half = T(0.5);
    const T* __restrict__ tb[6] = {ap.tau[0], ap.tau[1], ap.tau[2], ap.tau[3], ap.tau[4], ap.tau[5]};
    auto xd = [&](const Vec<T, VX>& f) { return xdiff<T, VX>(f, T(0), lane, last, false, 63); };

    // uv-node strain of a plane from rows of u and v there and w below/above
    auto uv_strain = [&](const Row3<T, VX>& U, const Row3<T, VX>& V, const Vec<T, VX>& wlo,
                         const Vec<T, VX>& whi, Vec<T, VX> s[4]) {
        const Vec<T, VX> dxu = xd(U.c), dxv = xd(V.c);
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
                        const Vec<T, VX>& vlo, const Row3<T, VX>& W, Vec<T, VX> s[2]) {
        const Vec<T, VX> dxw = xd(W.c);
#pragma unroll
        for (int e = 0; e < VX; ++e) {
            s[0].v[e] = half * ((uhi.v[e] - ulo.v[e]) * a.cz + dxw.v[e] * a.cx);
            s[1].v[e] = half * ((vhi.v[e] - vlo.v[e]) * a.cz + (W.p.v[e] - W.m.v[e]) * a.cy);
        }
    };

    // march state at plane ks (one below the chunk): uv strain of ks-1, w
    // strain of ks, w at ks
    const int ks = kb > 0 ? kb - 1 : 0;
    const int kend = ke < nz ? ke : nz - 1;              // last plane marched
    Vec<T, VX> P[4], Wst[2], wc;
    {
        constexpr unsigned S = sizeof(T);
        const unsigned p0 = (unsigned)(ks - kbase) * (unsigned)plane;
        const Row3<T, VX> Wk = load3<T, VX>(sl.w, p0, rm, r0, rp, xo);
        const Vec<T, VX> uk = bload<T, VX>(sl.u, xo, (p0 + r0) * S),
                         vk = bload<T, VX>(sl.v, xo, (p0 + r0) * S);
        if (ks > 0) {
            const unsigned pb = p0 - (unsigned)plane;          // ks - 1 >= kbase
            const Row3<T, VX> Ub = load3<T, VX>(sl.u, pb, rm, r0, rp, xo);
            const Row3<T, VX> Vb = load3<T, VX>(sl.v, pb, rm, r0, rp, xo);
            const Vec<T, VX> wb = bload<T, VX>(sl.w, xo, (pb + r0) * S);
            uv_strain(Ub, Vb, wb, Wk.c, P);
            w_strain(uk, Ub.c, vk, Vb.c, Wk, Wst);
        } else {
#pragma unroll
            for (int c = 0; c < 4; ++c) P[c] = vzero<T, VX>();
            w_strain(uk, vzero<T, VX>(), vk, vzero<T, VX>(), Wk, Wst);
        }
        wc = Wk.c;
    }
    // divergence state: the previous plane's stresses of this row and class bytes
    Vec<T, VX> xx_p = vzero<T, VX>(), xy_p = vzero<T, VX>(), xz_p = vzero<T, VX>(),
               yz_p = vzero<T, VX>(), zz_p = vzero<T, VX>();
    uint32_t m_p[VX];
#pragma unroll
    for (int e = 0; e < VX; ++e) m_p[e] = 0;
    Acc s0 = Acc(0), s1 = Acc(0), s2 = Acc(0);
    // the plane's loads go out one plane ahead: right after the barrier, so
    // they are in flight while the divergence of the plane is formed
    // (PF = 2: plane k+2's loads go out before plane k's arithmetic)
    PlaneIn<T, VX> in, in2;
    load_plane<T, VX>(a, sl, ks, kbase, rm, r0, rp, x, in);
    if constexpr (PF == 2)
        if (ks + 1 <= kend) load_plane<T, VX>(a, sl, ks + 1, kbase, rm, r0, rp, x, in2);
    for (int k = ks; k <= kend; ++k) {
        const bool up = k + 1 < nz;
        const int row = k * plane + r0;                  // uniform; the lane adds x
        const PlaneIn<T, VX> cur = in;
        if constexpr (PF == 2) {
            in = in2;
            if (k + 2 <= kend) load_plane<T, VX>(a, sl, k + 2, kbase, rm, r0, rp, x, in2);
        }
        const Row3<T, VX>& U = cur.U;
        const Row3<T, VX>& V = cur.V;
        const Row3<T, VX>& Wn = cur.Wn;
        const Vec<T, VX> un = cur.un, vn = cur.vn, pu = cur.pu, pw = cur.pw, lz = cur.lz;
        uint32_t m[VX];
#pragma unroll
        for (int e = 0; e < VX; ++e) m[e] = cur.m[e];
        // ---- strain: uv nodes of plane k, w nodes of plane k+1
        Vec<T, VX> S[4], N[2];
        uv_strain(U, V, wc, Wn.c, S);
        if (up) {
            w_strain(un, U.c, vn, V.c, Wn, N);
        } else {
            N[0] = N[1] = vzero<T, VX>();
        }
        // ---- stress: Smagorinsky, or the band value, or 0 in the body
        Vec<T, VX> t[6];
#pragma unroll
        for (int e = 0; e < VX; ++e) {
            const T z0 = a.log_z0 ? T(exp((double)lz.v[e])) : a.z0;
            const T s13 = half * (Wst[0].v[e] + N[0].v[e]);
            const T s23 = half * (Wst[1].v[e] + N[1].v[e]);
            const T ss = S[0].v[e] * S[0].v[e] + S[1].v[e] * S[1].v[e] + S[2].v[e] * S[2].v[e] +
                         T(2) * (S[3].v[e] * S[3].v[e] + s13 * s13 + s23 * s23);
            const T nu = mixing_sq(a, pu.v[e], z0) * sqrt_fast(T(2) * ss);
#pragma unroll
            for (int c = 0; c < 4; ++c) t[c].v[e] = T(-2) * nu * S[c].v[e];
            T mm[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) mm[c] = half * (P[c].v[e] + S[c].v[e]);
            const T sw = mm[0] * mm[0] + mm[1] * mm[1] + mm[2] * mm[2] +
                         T(2) * (mm[3] * mm[3] + Wst[0].v[e] * Wst[0].v[e] + Wst[1].v[e] * Wst[1].v[e]);
            const T nuw = mixing_sq(a, pw.v[e], z0) * sqrt_fast(T(2) * sw);
            t[4].v[e] = T(-2) * nuw * Wst[0].v[e];
            t[5].v[e] = T(-2) * nuw * Wst[1].v[e];
            const uint32_t cuv = m[e] & 3u, cw = (m[e] >> 2) & 3u;
            if (cuv == 1u) {
#pragma unroll
                for (int c = 0; c < 4; ++c) t[c].v[e] = tb[c][row + x + e];
            } else if (cuv == 2u) {
#pragma unroll
                for (int c = 0; c < 4; ++c) t[c].v[e] = T(0);
            }
            if (cw == 1u) {
                t[4].v[e] = tb[4][row + x + e];
                t[5].v[e] = tb[5][row + x + e];
            } else if (cw == 2u) {
                t[4].v[e] = t[5].v[e] = T(0);
            }
        }
        // ---- share the y-differenced components of plane k
        const int b = k % 3, bp = (k + 2) % 3;
#pragma unroll
        for (int e = 0; e < VX; ++e) {
            sh[b][0][wv][VX * lane + e] = t[3].v[e];
            sh[b][1][wv][VX * lane + e] = t[1].v[e];
            sh[b][2][wv][VX * lane + e] = t[5].v[e];
        }
        __syncthreads();
        if constexpr (PF == 1)
            if (k < kend) load_plane<T, VX>(a, sl, k + 1, kbase, rm, r0, rp, x, in);
        const Vec<T, VX> dxz = xd(t[4]), dxx_p = xd(xx_p), dxy_p = xd(xy_p);
        const bool zout = k >= kb && k < ke, xyout = k >= 1 && k - 1 >= kb && k - 1 < ke;
        if (row_out) {
            bool all = true;
#pragma unroll
            for (int e = 0; e < VX; ++e) all = all && outn[e];
            if (zout) {
                // w divergence of plane k
                Vec<T, VX> dz;
#pragma unroll
                for (int e = 0; e < VX; ++e) {
                    const int n = VX * lane + e;
                    const T dyz = sh[b][2][wv + 1][n] - sh[b][2][wv - 1][n];
                    dz.v[e] = dxz.v[e] * a.cx + dyz * a.cy + (t[2].v[e] - zz_p.v[e]) * a.cz;
                    if (outn[e] && !(m[e] & 32u)) s2 += (Acc)dz.v[e];
                }
                if (all) {
                    vstore_nt<T, VX>(ap.div[2] + row + x, dz);
                } else {
#pragma unroll
                    for (int e = 0; e < VX; ++e)
                        if (outn[e]) ap.div[2][row + x + e] = dz.v[e];
                }
            }
            if (xyout) {
                // uv divergence of plane k-1 (tau_xz, tau_yz of w planes k-1 and k)
                Vec<T, VX> dx, dy;
#pragma unroll
                for (int e = 0; e < VX; ++e) {
                    const int n = VX * lane + e;
                    dx.v[e] = dxx_p.v[e] * a.cx + (sh[bp][0][wv + 1][n] - sh[bp][0][wv - 1][n]) * a.cy +
                              (t[4].v[e] - xz_p.v[e]) * a.cz;
                    dy.v[e] = dxy_p.v[e] * a.cx + (sh[bp][1][wv + 1][n] - sh[bp][1][wv - 1][n]) * a.cy +
                              (t[5].v[e] - yz_p.v[e]) * a.cz;
                    if (outn[e] && !(m_p[e] & 16u)) {
                        s0 += (Acc)dx.v[e];
                        s1 += (Acc)dy.v[e];
                    }
                }
                const int rowp = row - plane;
                if (all) {
                    vstore_nt<T, VX>(ap.div[0] + rowp + x, dx);
                    vstore_nt<T, VX>(ap.div[1] + rowp + x, dy);
                } else {
#pragma unroll
                    for (int e = 0; e < VX; ++e) {
                        if (!outn[e]) continue;
                        ap.div[0][rowp + x + e] = dx.v[e];
                        ap.div[1][rowp + x + e] = dy.v[e];
                    }
                }
            }
        }
        // ---- carry upward
        xx_p = t[0];
        xy_p = t[3];
        xz_p = t[4];
        yz_p = t[5];
        zz_p = t[2];
#pragma unroll
        for (int e = 0; e < VX; ++e) m_p[e] = m[e];
#pragma unroll
        for (int c = 0; c < 4; ++c) P[c] = S[c];
        Wst[0] = N[0];
        Wst[1] = N[1];
        wc = Wn.c;
    }
    if (ke == nz) {
        // uv divergence of the top plane: tau_xz, tau_yz above it are 0
        const Vec<T, VX> dxx_p = xd(xx_p), dxy_p = xd(xy_p);
        const int bp = (nz - 1) % 3;
        const int rowt = (nz - 1) * plane + r0;
#pragma unroll
        for (int e = 0; e < VX; ++e) {
            if (!outn[e]) continue;
            const int n = VX * lane + e;
            const T dx = dxx_p.v[e] * a.cx + (sh[bp][0][wv + 1][n] - sh[bp][0][wv - 1][n]) * a.cy +
                         (T(0) - xz_p.v[e]) * a.cz;
            const T dy = dxy_p.v[e] * a.cx + (sh[bp][1][wv + 1][n] - sh[bp][1][wv - 1][n]) * a.cy +
                         (T(0) - yz_p.v[e]) * a.cz;
            ap.div[0][rowt + x + e] = dx;
            ap.div[1][rowt + x + e] = dy;
            if (!(m_p[e] & 16u)) {
                s0 += (Acc)dx;
                s1 += (Acc)dy;
            }
        }
    }
    if (!ap.drag) return;
    const double d0 = wave_sum((double)s0), d1 = wave_sum((double)s1), d2 = wave_sum((double)s2);
    if (lane == 0) {
        red[0][wv] = d0;
        red[1][wv] = d1;
        red[2][wv] = d2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double r = 0.0;
        for (int w = 0; w < kWaves; ++w) r += red[threadIdx.x][w];
        ap.partials[3L * lb + threadIdx.x] = r;
    }
}

__global__ void __launch_bounds__(256) k_sgs_apply_finalize(const double* __restrict__ p,
                                                            long nslots, double scale,
                                                            double* __restrict__ out) {
    finalize_slots(p, nslots, 3, 0u, scale, out);
}

// Planes per block: kChunk, fewer where a block's slab (its planes, two below
// and one above) would pass 4 GiB; below 1 when a single plane is that large.
int chunk_planes(const ibm_ctx* c) {
    const double plane_bytes = (double)c->g.nx * c->g.ny * (c->dtype == IBM_F64 ? 8 : 4);
    const double fit = std::floor(4294967295.0 / plane_bytes) - 4;
    return (int)std::min<double>(kChunk, fit);
}

template <typename T>
int sgs_apply_t(ibm_ctx* c, const T* phi_uv, const T* phi_w, const T* u, const T* v, const T* w,
                double z0, const T* log_z0, double cs, double kappa, const void* const tau[6],
                void* const ustar[3], const void* const gradp[3], double dt, void* const div[3],
                double* drag, hipStream_t s) {
    FusedArgs<T> a;
    a.u = u;
    a.v = v;
    a.w = w;
    a.phi_uv = phi_uv;
    a.phi_w = phi_w;
    a.log_z0 = log_z0;
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
    const int sp = span<1>();
    a.nxs = (c->g.nx + sp - 1) / sp;
    a.njb = (c->g.ny + kRows - 1) / kRows;
    a.kc = chunk_planes(c);
    if (a.kc < 1)
        return fail(IBM_E_ARG, "apply_sgs: an x-y plane of %ld nodes passes the 4 GiB reach of "
                    "the fused pass's 32-bit offsets", (long)a.plane);
    a.nblocks = (int)((long)a.nxs * a.njb * ((c->g.nz + a.kc - 1) / a.kc));
    a.per_xcd = (a.nblocks + 7) / 8;
    a.ap = make_apply_args<T>(c, c->cfg, tau, ustar, gradp, dt, div, drag);
    if (c->ap_cap < 3L * a.nblocks) return fail(IBM_E_STATE, "apply_sgs: reduction slots not sized");
    a.ap.partials = c->ap_partials;
    a.ap.nfblocks = (int)std::min<long>((4 * c->nfsegs + 7) / 8 * 8, 2048);
    const unsigned grid = (unsigned)(8 * a.per_xcd + a.ap.nfblocks);
    const bool wide = c->precision == IBM_PREC_MIXED || sizeof(T) == 8;   // drag in double
    const dim3 g3(grid), b3(64 * kWaves);
    // One node per lane.  In float the loads go out two planes ahead; in
    // double the third plane's registers would spill.  (Two nodes per lane
    // needed more registers than four waves per SIMD allow and measured
    // slower.)
    if constexpr (sizeof(T) == 4) {
        if (wide) hipLaunchKernelGGL((k_sgs_apply<T, double, 1, 2>), g3, b3, 0, s, a);
        else hipLaunchKernelGGL((k_sgs_apply<T, T, 1, 2>), g3, b3, 0, s, a);
    } else {
        hipLaunchKernelGGL((k_sgs_apply<T, double, 1, 1>), g3, b3, 0, s, a);
    }
    if (drag)
        hipLaunchKernelGGL(k_sgs_apply_finalize, dim3(1), dim3(256), 0, s,
                           (const double*)a.ap.partials, (long)a.nblocks, a.ap.dv, drag);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

}  // namespace

long sgs_apply_blocks(const ibm_ctx* c) {
    // the most blocks either node width can take (one node per lane)
    const int kc = std::max(chunk_planes(c), 1);
    return (long)((c->g.nx + span<1>() - 1) / span<1>()) * ((c->g.ny + kRows - 1) / kRows) *
           ((c->g.nz + kc - 1) / kc);
}

int launch_sgs_apply(ibm_ctx* c, const void* phi_uv, const void* phi_w, const void* u,
                     const void* v, const void* w, double z0, const void* log_z0, double cs,
                     double kappa, const void* const tau[6], void* const ustar[3],
                     const void* const gradp[3], double dt, void* const div[3], double* drag,
                     hipStream_t s) {
    if (c->dtype == IBM_F64)
        return sgs_apply_t<double>(c, (const double*)phi_uv, (const double*)phi_w,
                                   (const double*)u, (const double*)v, (const double*)w, z0,
                                   (const double*)log_z0, cs, kappa, tau, ustar, gradp, dt, div,
                                   drag, s);
    return sgs_apply_t<float>(c, (const float*)phi_uv, (const float*)phi_w, (const float*)u,
                              (const float*)v, (const float*)w, z0, (const float*)log_z0, cs, kappa,
                              tau, ustar, gradp, dt, div, drag, s);
}

}  // namespace ibm
