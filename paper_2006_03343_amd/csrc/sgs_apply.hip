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
// and a chunk of kz planes.  Wave wv computes the stress of row j0-1+wv (the
// two outer waves: the y halo) on 64 * VX consecutive nodes, the segment and
// H nodes on either side (H = max(2, VX)), exactly as the Smagorinsky kernel
// does for one row.  The strain, and with it the stress, is wrong on the
// outermost node of each side, which no output needs: x differences come
// from the adjacent lanes without edge loads.  Per plane the components
// differenced in y (tau_xy, tau_yy on uv nodes, tau_yz on w nodes) go
// through LDS (three plane buffers, so one barrier per plane suffices), z
// differences stay in registers.  The uv divergence of plane k needs tau_xz,
// tau_yz on w plane k+1, which the march reaches one plane later, so it is
// formed one plane behind the w divergence; a chunk starts one plane below
// its first (the march state rebuilt from the velocities there) and, unless
// it is the top one, ends one plane above its last.
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
constexpr int kChunk = 32;           // planes per block

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
    int nblocks;             // dense blocks (nxs * njb * z chunks)
    int per_xcd;             // logical dense blocks per XCD
    ApplyArgs<T> ap;         // tau (band values), ustar, gradp, div, mask, forcing segments, drag
};

// lambda^2 of eq. smag-1 (n = 2)
template <typename T>
__device__ inline T mixing_sq(const FusedArgs<T>& a, T d, T z0) {
    const T s = d + z0;
    if (!(s > T(0))) return T(0);
    const T wl = a.kappa * s;
    return T(1) / (a.inv_l0sq + T(1) / (wl * wl));
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

template <typename T, int VX>
__device__ inline Row3<T, VX> load3(const T* __restrict__ f, int pk, int rm, int r0, int rp, int x) {
    Row3<T, VX> r;
    r.m = vload<T, VX>(f + pk + rm + x);
    r.c = vload<T, VX>(f + pk + r0 + x);
    r.p = vload<T, VX>(f + pk + rp + x);
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
__device__ inline void load_plane(const FusedArgs<T>& a, int k, int rm, int r0, int rp, int x,
                                  PlaneIn<T, VX>& in) {
    const int pk = k * a.plane, q = pk + r0 + x;
    const bool up = k + 1 < a.nz;
    in.U = load3<T, VX>(a.u, pk, rm, r0, rp, x);
    in.V = load3<T, VX>(a.v, pk, rm, r0, rp, x);
    in.Wn = up ? load3<T, VX>(a.w, pk + a.plane, rm, r0, rp, x) : zero3<T, VX>();
    in.un = up ? vload<T, VX>(a.u + q + a.plane) : vzero<T, VX>();
    in.vn = up ? vload<T, VX>(a.v + q + a.plane) : vzero<T, VX>();
    in.pu = vload<T, VX>(a.phi_uv + q);
    in.pw = vload<T, VX>(a.phi_w + q);
    in.lz = a.log_z0 ? vload<T, VX>(a.log_z0 + q) : vzero<T, VX>();
    if constexpr (VX == 2) {
        const uint32_t two = *reinterpret_cast<const uint16_t*>(a.ap.mask + q);   // q is even
        in.m[0] = two & 0xffu;
        in.m[1] = two >> 8;
    } else {
#pragma unroll
        for (int e = 0; e < VX; ++e) in.m[e] = a.ap.mask[q + e];
    }
}

template <typename T, typename Acc, int VX>
__global__ void __launch_bounds__(64 * kWaves) k_sgs_apply(FusedArgs<T> a) {
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
    const int jb = t2 % a.njb, kc = t2 / a.njb;
    const int kb = kc * kChunk, ke = min(kb + kChunk, nz);
    const int x0 = xs * SPAN;
    const int jr = jb * kRows - 1 + wv;                  // this wave's row, unwrapped
    const int j = wrap(jr, ny);
    const int xb = x0 - H + VX * lane;                   // this lane's first node, unwrapped
    const int x = wrap(xb, nx);                          // nx % VX == 0: no wrap inside the lane
    const bool row_out = wv >= 1 && wv <= kRows && jr < ny;
    bool outn[VX];
#pragma unroll
    for (int e = 0; e < VX; ++e) outn[e] = row_out && xb + e >= x0 && xb + e < min(x0 + SPAN, nx);
    const int rm = wrap(j - 1, ny) * nx, r0 = j * nx, rp = wrap(j + 1, ny) * nx;
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
        const int p0 = ks * plane;
        const Row3<T, VX> Wk = load3<T, VX>(a.w, p0, rm, r0, rp, x);
        const Vec<T, VX> uk = vload<T, VX>(a.u + p0 + r0 + x), vk = vload<T, VX>(a.v + p0 + r0 + x);
        if (ks > 0) {
            const int pb = p0 - plane;
            const Row3<T, VX> Ub = load3<T, VX>(a.u, pb, rm, r0, rp, x);
            const Row3<T, VX> Vb = load3<T, VX>(a.v, pb, rm, r0, rp, x);
            const Vec<T, VX> wb = vload<T, VX>(a.w + pb + r0 + x);
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
    PlaneIn<T, VX> in;
    load_plane<T, VX>(a, ks, rm, r0, rp, x, in);
    for (int k = ks; k <= kend; ++k) {
        const bool up = k + 1 < nz;
        const int q = k * plane + r0 + x;
        const Row3<T, VX>& U = in.U;
        const Row3<T, VX>& V = in.V;
        const Row3<T, VX> Wn = in.Wn;
        const Vec<T, VX> un = in.un, vn = in.vn, pu = in.pu, pw = in.pw, lz = in.lz;
        uint32_t m[VX];
#pragma unroll
        for (int e = 0; e < VX; ++e) m[e] = in.m[e];
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
            const T nu = mixing_sq(a, pu.v[e], z0) * sqrt(T(2) * ss);
#pragma unroll
            for (int c = 0; c < 4; ++c) t[c].v[e] = T(-2) * nu * S[c].v[e];
            T mm[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) mm[c] = half * (P[c].v[e] + S[c].v[e]);
            const T sw = mm[0] * mm[0] + mm[1] * mm[1] + mm[2] * mm[2] +
                         T(2) * (mm[3] * mm[3] + Wst[0].v[e] * Wst[0].v[e] + Wst[1].v[e] * Wst[1].v[e]);
            const T nuw = mixing_sq(a, pw.v[e], z0) * sqrt(T(2) * sw);
            t[4].v[e] = T(-2) * nuw * Wst[0].v[e];
            t[5].v[e] = T(-2) * nuw * Wst[1].v[e];
            const uint32_t cuv = m[e] & 3u, cw = (m[e] >> 2) & 3u;
            if (cuv == 1u) {
#pragma unroll
                for (int c = 0; c < 4; ++c) t[c].v[e] = tb[c][q + e];
            } else if (cuv == 2u) {
#pragma unroll
                for (int c = 0; c < 4; ++c) t[c].v[e] = T(0);
            }
            if (cw == 1u) {
                t[4].v[e] = tb[4][q + e];
                t[5].v[e] = tb[5][q + e];
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
        if (k < kend) load_plane<T, VX>(a, k + 1, rm, r0, rp, x, in);
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
                    vstore_nt<T, VX>(ap.div[2] + q, dz);
                } else {
#pragma unroll
                    for (int e = 0; e < VX; ++e)
                        if (outn[e]) ap.div[2][q + e] = dz.v[e];
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
                const int qp = q - plane;
                if (all) {
                    vstore_nt<T, VX>(ap.div[0] + qp, dx);
                    vstore_nt<T, VX>(ap.div[1] + qp, dy);
                } else {
#pragma unroll
                    for (int e = 0; e < VX; ++e) {
                        if (!outn[e]) continue;
                        ap.div[0][qp + e] = dx.v[e];
                        ap.div[1][qp + e] = dy.v[e];
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
        const int qt = (nz - 1) * plane + r0 + x;
#pragma unroll
        for (int e = 0; e < VX; ++e) {
            if (!outn[e]) continue;
            const int n = VX * lane + e;
            const T dx = dxx_p.v[e] * a.cx + (sh[bp][0][wv + 1][n] - sh[bp][0][wv - 1][n]) * a.cy +
                         (T(0) - xz_p.v[e]) * a.cz;
            const T dy = dxy_p.v[e] * a.cx + (sh[bp][1][wv + 1][n] - sh[bp][1][wv - 1][n]) * a.cy +
                         (T(0) - yz_p.v[e]) * a.cz;
            ap.div[0][qt + e] = dx;
            ap.div[1][qt + e] = dy;
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
    // two nodes per lane (float: in double the registers would spill) when no
    // lane's pair straddles the periodic end and every field allows 8-byte
    // access
    bool pair = sizeof(T) == 4 && c->g.nx % 2 == 0;
    for (const void* p : {(const void*)phi_uv, (const void*)phi_w, (const void*)u, (const void*)v,
                          (const void*)w, (const void*)log_z0})
        pair = pair && (!p || (uintptr_t)p % (2 * sizeof(T)) == 0);
    for (int i = 0; i < 6; ++i) pair = pair && (uintptr_t)tau[i] % (2 * sizeof(T)) == 0;
    for (int i = 0; i < 3; ++i) pair = pair && (uintptr_t)div[i] % (2 * sizeof(T)) == 0;
    const int sp = pair ? span<2>() : span<1>();
    a.nxs = (c->g.nx + sp - 1) / sp;
    a.njb = (c->g.ny + kRows - 1) / kRows;
    a.nblocks = (int)((long)a.nxs * a.njb * ((c->g.nz + kChunk - 1) / kChunk));
    a.per_xcd = (a.nblocks + 7) / 8;
    a.ap = make_apply_args<T>(c, c->cfg, tau, ustar, gradp, dt, div, drag);
    if (c->ap_cap < 3L * a.nblocks) return fail(IBM_E_STATE, "apply_sgs: reduction slots not sized");
    a.ap.partials = c->ap_partials;
    a.ap.nfblocks = (int)std::min<long>((4 * c->nfsegs + 7) / 8 * 8, 2048);
    const unsigned grid = (unsigned)(8 * a.per_xcd + a.ap.nfblocks);
    const bool wide = c->precision == IBM_PREC_MIXED || sizeof(T) == 8;   // drag in double
    const dim3 g3(grid), b3(64 * kWaves);
    if constexpr (sizeof(T) == 4) {
        if (pair && wide) hipLaunchKernelGGL((k_sgs_apply<T, double, 2>), g3, b3, 0, s, a);
        else if (pair) hipLaunchKernelGGL((k_sgs_apply<T, T, 2>), g3, b3, 0, s, a);
        else if (wide) hipLaunchKernelGGL((k_sgs_apply<T, double, 1>), g3, b3, 0, s, a);
        else hipLaunchKernelGGL((k_sgs_apply<T, T, 1>), g3, b3, 0, s, a);
    } else {
        hipLaunchKernelGGL((k_sgs_apply<T, double, 1>), g3, b3, 0, s, a);
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
    return (long)((c->g.nx + span<1>() - 1) / span<1>()) * ((c->g.ny + kRows - 1) / kRows) *
           ((c->g.nz + kChunk - 1) / kChunk);
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
