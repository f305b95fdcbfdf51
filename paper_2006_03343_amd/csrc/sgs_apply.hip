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
// A block of kWaves waves owns kRows rows j0 .. j0+kRows-1 of a 62-node x
// segment and marches up the whole column.  Wave wv computes the stress of row
// j0-1+wv (the two outer waves: the y halo) for 64 nodes x0-1 .. x0+62 (lanes
// 0 and 63: the x halo), exactly as the Smagorinsky kernel does for one row;
// per plane the components that are differenced in y (tau_xy, tau_yy on uv
// nodes, tau_yz on w nodes) go through LDS (three plane buffers, so one
// barrier per plane suffices), x differences come from the adjacent lanes, z
// differences from registers.  The uv divergence of plane k needs tau_xz,
// tau_yz on w plane k+1, which the march reaches one plane later, so it is
// formed one plane behind the w divergence.
//
// Bytes per node: u, v, w, phi_uv, phi_w (log z0) in, the class byte, the
// band stress where there is one, div out; the halo rows and columns of a
// block are the interior rows of its neighbours (L2).
#include <algorithm>
#include <cmath>

#include "kernels.h"

// Every product and sum rounded as written, as in the Smagorinsky kernel.
#pragma clang fp contract(off)

namespace ibm {
namespace {

constexpr int kRows = 4;             // divergence rows per block
constexpr int kWaves = kRows + 2;    // one stress row per wave: rows j0-1 .. j0+kRows
constexpr int kSpan = 62;            // x nodes per block written (lanes 1 .. 62)

template <typename T>
struct FusedArgs {
    const T *u, *v, *w, *phi_uv, *phi_w, *log_z0;
    int nx, ny, nz, plane;
    T cx, cy, cz;            // 1/(2 dx), 1/(2 dy), 1/dz
    T inv_l0sq;              // 1 / lambda_0^2
    T kappa, z0;
    int nxs;                 // x segments
    int nblocks;             // dense blocks (nxs * row blocks)
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

template <typename T>
__device__ inline int wrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// f[x+1] - f[x-1] from the adjacent lanes (valid on lanes 1 .. 62).
template <typename T>
__device__ inline T lane_diff(T f) {
    return __shfl_down(f, 1, 64) - __shfl_up(f, 1, 64);
}

// One row (three rows of the field for the y difference) and, for lanes 0
// and 1, the values left of lane 0 and right of lane 63.
template <typename T>
struct Row3 {
    Vec<T, 1> m, c, p;
    T e;
};

template <typename T>
__device__ inline Row3<T> load3(const T* __restrict__ f, int pk, int rm, int r0, int rp, int x,
                                int ex) {
    Row3<T> r;
    r.m.v[0] = f[pk + rm + x];
    r.c.v[0] = f[pk + r0 + x];
    r.p.v[0] = f[pk + rp + x];
    r.e = f[pk + r0 + ex];
    return r;
}

template <typename T>
__device__ inline Row3<T> zero3() {
    Row3<T> r;
    r.m.v[0] = r.c.v[0] = r.p.v[0] = T(0);
    r.e = T(0);
    return r;
}

template <typename T, typename Acc>
__global__ void __launch_bounds__(64 * kWaves) k_sgs_apply(FusedArgs<T> a) {
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
    __shared__ T sh[3][3][kWaves][64];                   // [plane % 3][xy, yy, yz][row][lane]
    __shared__ double red[3][kWaves];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nx = a.nx, ny = a.ny, nz = a.nz, plane = a.plane;
    const int xs = lb % a.nxs, jb = lb / a.nxs;
    const int x0 = xs * kSpan;
    const int jr = jb * kRows - 1 + wv;                  // this wave's row, unwrapped
    const int j = wrap<T>(jr, ny);
    const int xn = x0 - 1 + lane;                        // this lane's node, unwrapped
    const int x = wrap<T>(xn, nx);
    const int ex = wrap<T>((lane & 1) ? x0 + 63 : x0 - 2, nx);   // left of lane 0, right of lane 63
    const bool out = wv >= 1 && wv <= kRows && jr < ny && lane >= 1 && lane <= kSpan && xn < nx;
    const int rm = wrap<T>(j - 1, ny) * nx, r0 = j * nx, rp = wrap<T>(j + 1, ny) * nx;
    const bool last = lane == 63;
    const T half = T(0.5);
    const T* __restrict__ tb[6] = {ap.tau[0], ap.tau[1], ap.tau[2], ap.tau[3], ap.tau[4], ap.tau[5]};

    // uv-node strain of a plane from rows of u and v there and w below/above
    auto uv_strain = [&](const Row3<T>& U, const Row3<T>& V, T wlo, T whi, T s[4]) {
        const T dxu = xdiff<T, 1>(U.c, U.e, lane, last, false, 63).v[0];
        const T dxv = xdiff<T, 1>(V.c, V.e, lane, last, false, 63).v[0];
        s[0] = dxu * a.cx;
        s[1] = (V.p.v[0] - V.m.v[0]) * a.cy;
        s[2] = (whi - wlo) * a.cz;
        s[3] = half * ((U.p.v[0] - U.m.v[0]) * a.cy + dxv * a.cx);
    };
    // w-node strain of a plane from u, v at the uv planes above and below it
    // and rows of w there
    auto w_strain = [&](T uhi, T ulo, T vhi, T vlo, const Row3<T>& W, T s[2]) {
        const T dxw = xdiff<T, 1>(W.c, W.e, lane, last, false, 63).v[0];
        s[0] = half * ((uhi - ulo) * a.cz + dxw * a.cx);
        s[1] = half * ((vhi - vlo) * a.cz + (W.p.v[0] - W.m.v[0]) * a.cy);
    };

    // march state: uv strain of plane k-1, w strain of plane k, w at plane k
    T P[4] = {T(0), T(0), T(0), T(0)}, Wst[2], wc;
    {
        const Row3<T> Wk = load3(a.w, 0, rm, r0, rp, x, ex);
        w_strain(a.u[r0 + x], T(0), a.v[r0 + x], T(0), Wk, Wst);
        wc = Wk.c.v[0];
    }
    // divergence state: the previous plane's stresses of this row and class byte
    T xx_p = T(0), xy_p = T(0), xz_p = T(0), yz_p = T(0), zz_p = T(0);
    uint32_t m_p = 0;
    Acc s0 = Acc(0), s1 = Acc(0), s2 = Acc(0);
    for (int k = 0; k < nz; ++k) {
        const int pk = k * plane;
        const bool up = k + 1 < nz;
        const int q = pk + r0 + x;
        // ---- every load of the plane
        const Row3<T> U = load3(a.u, pk, rm, r0, rp, x, ex);
        const Row3<T> V = load3(a.v, pk, rm, r0, rp, x, ex);
        const Row3<T> Wn = up ? load3(a.w, pk + plane, rm, r0, rp, x, ex) : zero3<T>();
        const T un = up ? a.u[q + plane] : T(0);
        const T vn = up ? a.v[q + plane] : T(0);
        const T pu = a.phi_uv[q], pw = a.phi_w[q];
        const T lz = a.log_z0 ? a.log_z0[q] : T(0);
        const uint32_t m = ap.mask[q];
        // ---- strain: uv nodes of plane k, w nodes of plane k+1
        T S[4], N[2] = {T(0), T(0)};
        uv_strain(U, V, wc, Wn.c.v[0], S);
        if (up) w_strain(un, U.c.v[0], vn, V.c.v[0], Wn, N);
        // ---- stress: Smagorinsky, or the band value, or 0 in the body
        T t[6];
        {
            const T z0 = a.log_z0 ? T(exp((double)lz)) : a.z0;
            const T s13 = half * (Wst[0] + N[0]);
            const T s23 = half * (Wst[1] + N[1]);
            const T ss = S[0] * S[0] + S[1] * S[1] + S[2] * S[2] +
                         T(2) * (S[3] * S[3] + s13 * s13 + s23 * s23);
            const T nu = mixing_sq(a, pu, z0) * sqrt(T(2) * ss);
#pragma unroll
            for (int c = 0; c < 4; ++c) t[c] = T(-2) * nu * S[c];
            T mm[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) mm[c] = half * (P[c] + S[c]);
            const T sw = mm[0] * mm[0] + mm[1] * mm[1] + mm[2] * mm[2] +
                         T(2) * (mm[3] * mm[3] + Wst[0] * Wst[0] + Wst[1] * Wst[1]);
            const T nuw = mixing_sq(a, pw, z0) * sqrt(T(2) * sw);
            t[4] = T(-2) * nuw * Wst[0];
            t[5] = T(-2) * nuw * Wst[1];
            const uint32_t cuv = m & 3u, cw = (m >> 2) & 3u;
            if (cuv == 1u) {
#pragma unroll
                for (int c = 0; c < 4; ++c) t[c] = tb[c][q];
            } else if (cuv == 2u) {
#pragma unroll
                for (int c = 0; c < 4; ++c) t[c] = T(0);
            }
            if (cw == 1u) {
                t[4] = tb[4][q];
                t[5] = tb[5][q];
            } else if (cw == 2u) {
                t[4] = t[5] = T(0);
            }
        }
        // ---- share the y-differenced components of plane k
        const int b = k % 3, bp = (k + 2) % 3;
        sh[b][0][wv][lane] = t[3];
        sh[b][1][wv][lane] = t[1];
        sh[b][2][wv][lane] = t[5];
        __syncthreads();
        const T dxz = lane_diff(t[4]);
        const T dxx_p = lane_diff(xx_p), dxy_p = lane_diff(xy_p);
        if (out) {
            // w divergence of plane k
            const T dyz = sh[b][2][wv + 1][lane] - sh[b][2][wv - 1][lane];
            const T dz = dxz * a.cx + dyz * a.cy + (t[2] - zz_p) * a.cz;
            ap.div[2][q] = dz;
            if (!(m & 32u)) s2 += (Acc)dz;
            if (k > 0) {
                // uv divergence of plane k-1 (tau_xz, tau_yz of w planes k-1 and k)
                const int qp = q - plane;
                const T dx = dxx_p * a.cx + (sh[bp][0][wv + 1][lane] - sh[bp][0][wv - 1][lane]) * a.cy +
                             (t[4] - xz_p) * a.cz;
                const T dy = dxy_p * a.cx + (sh[bp][1][wv + 1][lane] - sh[bp][1][wv - 1][lane]) * a.cy +
                             (t[5] - yz_p) * a.cz;
                ap.div[0][qp] = dx;
                ap.div[1][qp] = dy;
                if (!(m_p & 16u)) {
                    s0 += (Acc)dx;
                    s1 += (Acc)dy;
                }
            }
        }
        // ---- carry upward
        xx_p = t[0];
        xy_p = t[3];
        xz_p = t[4];
        yz_p = t[5];
        zz_p = t[2];
        m_p = m;
#pragma unroll
        for (int c = 0; c < 4; ++c) P[c] = S[c];
        Wst[0] = N[0];
        Wst[1] = N[1];
        wc = Wn.c.v[0];
    }
    {
        // uv divergence of the top plane: tau_xz, tau_yz above it are 0
        const T dxx_p = lane_diff(xx_p), dxy_p = lane_diff(xy_p);
        if (out) {
            const int bp = (nz - 1) % 3;
            const int qp = (nz - 1) * plane + r0 + x;
            const T dx = dxx_p * a.cx + (sh[bp][0][wv + 1][lane] - sh[bp][0][wv - 1][lane]) * a.cy +
                         (T(0) - xz_p) * a.cz;
            const T dy = dxy_p * a.cx + (sh[bp][1][wv + 1][lane] - sh[bp][1][wv - 1][lane]) * a.cy +
                         (T(0) - yz_p) * a.cz;
            ap.div[0][qp] = dx;
            ap.div[1][qp] = dy;
            if (!(m_p & 16u)) {
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
    a.nxs = (c->g.nx + kSpan - 1) / kSpan;
    a.nblocks = (int)sgs_apply_blocks(c);
    a.per_xcd = (a.nblocks + 7) / 8;
    a.ap = make_apply_args<T>(c, c->cfg, tau, ustar, gradp, dt, div, drag);
    if (c->ap_cap < 3L * a.nblocks) return fail(IBM_E_STATE, "apply_sgs: reduction slots not sized");
    a.ap.partials = c->ap_partials;
    a.ap.nfblocks = (int)std::min<long>((4 * c->nfsegs + 7) / 8 * 8, 2048);
    const unsigned grid = (unsigned)(8 * a.per_xcd + a.ap.nfblocks);
    if (c->precision == IBM_PREC_MIXED || sizeof(T) == 8)
        hipLaunchKernelGGL((k_sgs_apply<T, double>), dim3(grid), dim3(64 * kWaves), 0, s, a);
    else
        hipLaunchKernelGGL((k_sgs_apply<T, float>), dim3(grid), dim3(64 * kWaves), 0, s, a);
    if (drag)
        hipLaunchKernelGGL(k_sgs_apply_finalize, dim3(1), dim3(256), 0, s,
                           (const double*)a.ap.partials, (long)a.nblocks, a.ap.dv, drag);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

}  // namespace

long sgs_apply_blocks(const ibm_ctx* c) {
    return (long)((c->g.nx + kSpan - 1) / kSpan) * ((c->g.ny + kRows - 1) / kRows);
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
