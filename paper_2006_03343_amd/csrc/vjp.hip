// vjp.hip -- hand-written reverse mode of one stage pass.
//
// Forward (one velocity state u = u* that is sampled and forced):
//   tau_out = wall model at band nodes (depends on u through the sample and on
//             log z0), 0 at solid nodes, tau_sgs elsewhere;
//   div     = D tau_out;  drag_c = dV sum_{phi > 0} div_c;
//   ustar   = u where phi > 0, (3 dt / 2) grad p elsewhere.
// Reverse:
//   1. dense pass:  gu = g_ustar [phi_uv > 0] (and v, w alike); glog_z0 = 0;
//   2. band pass:   one thread per band node (its uv record, then its w
//                   record, so their log z0 cotangents add in a fixed order);
//                   per record the stress cotangent at its node,
//                   g_tau + (D^T gbar)(q) with gbar = g_div + dV g_drag [phi > 0],
//                   evaluated from the transposed stencil at that node only;
//                   then back through tau = -c |U_r| (U_r n^T + n U_r^T):
//                   U_r cotangent, projection (I - n n^T), and the log z0
//                   cotangent dc/dlog z0 = 2 kappa^2 / ln(phi_c / z0)^3;
//   3. gather pass: each velocity node touched by a sample stencil adds the
//                   weighted record cotangents, reading a transposed map sorted
//                   by node (built once per geometry, with each entry's
//                   trilinear weight) -- no atomics, so the result is
//                   deterministic; one launch for both node sets (uv-grid
//                   nodes first, then w-grid nodes), blocks of consecutive
//                   nodes staging their entries through LDS.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <climits>
#include <numeric>
#include <vector>

#include "device.h"
#include "ibm_impl.h"

namespace ibm {
namespace {

inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename T>
__global__ void k_vjp_dense(const T* __restrict__ g0, const T* __restrict__ g1,
                            const T* __restrict__ g2, const uint32_t* __restrict__ fmask, int nx,
                            long rows, int wrow, T* __restrict__ gu, T* __restrict__ gv,
                            T* __restrict__ gw, T* __restrict__ glz) {
    // launched in blocks of 256 over n < 2^31 nodes: 256 divides 2^31, so
    // every thread index, padding included, fits in an int
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= rows * nx) return;
    const int row = q / nx;
    const int x = q - row * nx;
    const uint32_t fb = fmask[row * wrow + (x >> 4)] >> (2 * (x & 15));
    gu[q] = (fb & 1u) ? T(0) : g0[q];
    gv[q] = (fb & 1u) ? T(0) : g1[q];
    gw[q] = (fb & 2u) ? T(0) : g2[q];
    if (glz) glz[q] = T(0);
}

template <typename T>
struct BandArgs {
    RecView<T> recs[2];        // uv records, w records
    const int32_t* brec;       // per band node: [uv record or -1, w record or -1]
    long nb;                   // band nodes
    long nuv;                  // uv records (the w records follow them in rbar)
    const T *u, *v, *w, *log_z0;
    const T* g_tau[6];         // with HAS_GT: g_div[0] in place of a null entry (never used)
    unsigned gt_mask;          // bit i: g_tau[i] was given
    const T* g_div[3];
    const uint32_t* fmask;
    int nx, ny, nz, wrow;
    long plane;
    double gdrag[3];
    double dv;
    T cx, cy, cz;
    double ln_scalar, ln_phic, kappa, dz;
    int mixed;
    T* rbar;                   // 3 x ntot
    long ntot;
    T* glz;                    // nullable
};

// Cotangent of div_c at node (ii, jj, k) (ii, jj already wrapped into the
// periodic range), including the drag term; zero outside 0 <= k < nz.  32-bit
// offsets: a context holds fewer than 2^31 nodes.
template <typename T>
__device__ inline T gbar(const BandArgs<T>& a, int c, int ii, int jj, int k) {
    // outside the planes the loads read plane 0 (in bounds) and the value is
    // dropped: no branch around the loads, so the compiler issues all of a
    // record's loads before waiting on any
    const bool in = k >= 0 && k < a.nz;
    const int row = (in ? k : 0) * a.ny + jj;
    const int q = row * a.nx + ii;
    const uint32_t fb = a.fmask[row * a.wrow + (ii >> 4)] >> (2 * (ii & 15));
    const bool forced = (c < 2) ? (fb & 1u) : (fb & 2u);
    T g = a.g_div[c][q];
    if (!forced) g += (T)(a.dv * a.gdrag[c]);
    return in ? g : T(0);
}

// f[off], f[off + sx]: one load of both where they are contiguous (sx = 1),
// two across the periodic seam (global loads of several dwords need only
// 4-byte alignment).
template <typename T>
__device__ inline void load_xpair(const T* __restrict__ f, int off, int sx, T& lo, T& hi) {
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

// Trilinear sample from the stencil's lower corners c00, c01 (the upper
// ones are c00 + sx, c01 + sx) at plane offsets z0, z1.
template <typename T>
__device__ inline T trilerp_xpair(const T* __restrict__ f, int c00, int c01, int sx, int z0,
                                  int z1, T fx, T fy, T fz) {
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
    return (a0 * gy + b0 * fy) * gz + (a1 * gy + b1 * fy) * fz;
}

// The reverse of one band record of node set ``kind``: writes its sample
// cotangent into rbar and returns its log z0 cotangent (0 without a field).
// The g_tau cotangent of component i at node q (0 without one): loaded
// unconditionally when any is given, so no branch separates the loads.
template <typename T, bool HAS_GT>
__device__ inline T gtau(const BandArgs<T>& a, int i, int q) {
    if constexpr (!HAS_GT) {
        return T(0);
    } else {
        const T g = a.g_tau[i][q];
        return (a.gt_mask >> i) & 1u ? g : T(0);
    }
}

template <typename T, bool HAS_LZ, bool HAS_GT>
__device__ inline T band_record(const BandArgs<T>& a, int kind, long r) {
    const RecView<T>& R = a.recs[kind];
    const int q = R.q[r];
    const int k = q / (int)a.plane;
    const int rem = q - k * (int)a.plane;
    const int j = rem / a.nx, i = rem - j * a.nx;
    const int im = i == 0 ? a.nx - 1 : i - 1, ip = i + 1 == a.nx ? 0 : i + 1;
    const int jm = j == 0 ? a.ny - 1 : j - 1, jp = j + 1 == a.ny ? 0 : j + 1;
    const T n0 = R.nx[r], n1 = R.ny[r], n2 = R.nz[r];
    const int base = R.base[r];
    const int sx = R.sx[r], c00 = base, c01 = base + R.sy[r];
    const T fx = R.fx[r], fy = R.fy[r];
    const int ku = R.ku[r], kw = R.kw[r];
    const int pl = (int)a.plane;
    const int zu0 = ku * pl, zu1 = min(ku + 1, a.nz - 1) * pl;
    const int zw0 = kw * pl, zw1 = min(kw + 1, a.nz - 1) * pl;
    const T us = trilerp_xpair<T>(a.u, c00, c01, sx, zu0, zu1, fx, fy, R.fzu[r]);
    const T vs = trilerp_xpair<T>(a.v, c00, c01, sx, zu0, zu1, fx, fy, R.fzu[r]);
    const T ws = trilerp_xpair<T>(a.w, c00, c01, sx, zw0, zw1, fx, fy, R.fzw[r]);
    const T un = us * n0 + vs * n1 + ws * n2;
    const T ur0 = us - un * n0, ur1 = vs - un * n1, ur2 = ws - un * n2;
    const T U = sqrt(ur0 * ur0 + ur1 * ur1 + ur2 * ur2);
    double lnr;
    if (HAS_LZ)
        lnr = a.ln_phic - (double)a.log_z0[q];
    else
        lnr = a.ln_scalar;
    T c;
    if (a.mixed && fabs((double)R.phi[r]) <= a.dz) {
        const double kl = a.kappa / lnr;
        c = (T)(kl * kl);
    } else {
        const T kl = T(a.kappa) / (HAS_LZ ? T(a.ln_phic) - a.log_z0[q] : T(a.ln_scalar));
        c = kl * kl;
    }
    // stress cotangent at this node for the components the record stores
    T S, P0, P1, P2;
    if (kind == IBM_GRID_UV) {
        const T txx = gtau<T, HAS_GT>(a, 0, q) -
                      (gbar(a, 0, ip, j, k) - gbar(a, 0, im, j, k)) * a.cx;
        const T tyy = gtau<T, HAS_GT>(a, 1, q) -
                      (gbar(a, 1, i, jp, k) - gbar(a, 1, i, jm, k)) * a.cy;
        const T tzz = gtau<T, HAS_GT>(a, 2, q) +
                      (gbar(a, 2, i, j, k) - gbar(a, 2, i, j, k + 1)) * a.cz;
        const T txy = gtau<T, HAS_GT>(a, 3, q) -
                      (gbar(a, 0, i, jp, k) - gbar(a, 0, i, jm, k)) * a.cy -
                      (gbar(a, 1, ip, j, k) - gbar(a, 1, im, j, k)) * a.cx;
        S = txx * (T(2) * ur0 * n0) + tyy * (T(2) * ur1 * n1) + tzz * (T(2) * ur2 * n2) +
            txy * (ur0 * n1 + n0 * ur1);
        P0 = txx * (T(2) * n0) + txy * n1;
        P1 = tyy * (T(2) * n1) + txy * n0;
        P2 = tzz * (T(2) * n2);
    } else {
        const T txz = gtau<T, HAS_GT>(a, 4, q) -
                      (gbar(a, 2, ip, j, k) - gbar(a, 2, im, j, k)) * a.cx +
                      (gbar(a, 0, i, j, k - 1) - gbar(a, 0, i, j, k)) * a.cz;
        const T tyz = gtau<T, HAS_GT>(a, 5, q) -
                      (gbar(a, 2, i, jp, k) - gbar(a, 2, i, jm, k)) * a.cy +
                      (gbar(a, 1, i, j, k - 1) - gbar(a, 1, i, j, k)) * a.cz;
        S = txz * (ur0 * n2 + n0 * ur2) + tyz * (ur1 * n2 + n1 * ur2);
        P0 = txz * n2;
        P1 = tyz * n2;
        P2 = txz * n0 + tyz * n1;
    }
    // tau = -c U M, M = U_r n^T + n U_r^T:  dtau/dU_r,j = -c (U_r,j / U M + U dM/dU_r,j)
    T b0 = T(0), b1 = T(0), b2 = T(0), gl = T(0);
    if (U > T(0)) {
        const T sU = S / U;
        b0 = -c * (ur0 * sU + U * P0);
        b1 = -c * (ur1 * sU + U * P1);
        b2 = -c * (ur2 * sU + U * P2);
        if (HAS_LZ) {
            const double cbar = -(double)U * (double)S;
            gl = (T)(cbar * 2.0 * a.kappa * a.kappa / (lnr * lnr * lnr));
        }
    }
    // through U_r = (I - n n^T) u_s
    const T bn = b0 * n0 + b1 * n1 + b2 * n2;
    const long rr = (kind ? a.nuv : 0) + r;
    a.rbar[rr] = b0 - bn * n0;
    a.rbar[a.ntot + rr] = b1 - bn * n1;
    a.rbar[2 * a.ntot + rr] = b2 - bn * n2;
    return gl;
}

// One thread per band node: its uv record, then its w record; the log z0
// cotangent of the node is 0 (the dense pass) + the uv record's + the w
// record's, in that order.
template <typename T, bool HAS_LZ, bool HAS_GT>
__global__ void __launch_bounds__(256) k_vjp_band(BandArgs<T> a) {
    const long b = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.nb) return;
    const int ruv = a.brec[2 * b], rw = a.brec[2 * b + 1];
    T gl = T(0);
    int q = 0;
    if (ruv >= 0) {
        gl = gl + band_record<T, HAS_LZ, HAS_GT>(a, IBM_GRID_UV, ruv);
        q = a.recs[0].q[ruv];
    }
    if (rw >= 0) {
        gl = gl + band_record<T, HAS_LZ, HAS_GT>(a, IBM_GRID_W, rw);
        q = a.recs[1].q[rw];
    }
    if (HAS_LZ && a.glz) a.glz[q] = gl;
}

template <typename T>
struct GatherArgs {
    long ntot;
    const int32_t *node[2], *off[2], *erec[2];
    const T* wgt[2];
    long m[2];
    int nb0;                   // blocks of the uv-grid nodes (u, v cotangents)
    const T* rbar;
    T* out0[2];                // gu (uv grid), gw (w grid)
    T* out1;                   // gv
};

// 256 consecutive touched nodes per block, the uv-grid nodes' blocks first.
// Their entries are contiguous in the map: the block stages them kChunk at a
// time -- each thread loads kPer entries (record, weight) and the record
// cotangents they point to, all issued before use, and leaves the weighted
// products in LDS -- then each thread adds its own node's products in entry
// order.  The entry reads are coalesced across the block instead of strided
// per node, and every node's sum keeps one fixed order (deterministic).
constexpr int kGatherBlock = 256;
constexpr int kGatherPer = 4;
constexpr int kGatherChunk = kGatherBlock * kGatherPer;

template <typename T>
__global__ void __launch_bounds__(kGatherBlock) k_vjp_gather(GatherArgs<T> ga) {
    __shared__ T p0s[kGatherChunk], p1s[kGatherChunk];
    __shared__ int offs[kGatherBlock + 1];
    const int zg = (int)blockIdx.x < ga.nb0 ? 0 : 1;
    const long m0 = (long)((int)blockIdx.x - (zg ? ga.nb0 : 0)) * kGatherBlock;
    const long mcount = min((long)kGatherBlock, ga.m[zg] - m0);
    const int t = threadIdx.x;
    const int32_t* __restrict__ off = ga.off[zg];
    const int32_t* __restrict__ erec = ga.erec[zg];
    const T* __restrict__ wgt = ga.wgt[zg];
    const T* __restrict__ rb0 = ga.rbar + (zg ? 2 * ga.ntot : 0);
    const T* __restrict__ rb1 = ga.rbar + ga.ntot;
    if (t < mcount) offs[t] = off[m0 + t];
    if (t == 0) offs[mcount] = off[m0 + mcount];      // the map holds m + 1 offsets
    __syncthreads();
    const int e0 = offs[0], e1 = offs[mcount];
    const int my0 = t < mcount ? offs[t] : e1, my1 = t < mcount ? offs[t + 1] : e1;
    T s0 = T(0), s1 = T(0);
    for (int cb = e0; cb < e1; cb += kGatherChunk) {
        const int ce = min(cb + kGatherChunk, e1);
        int rr[kGatherPer];
        T wg[kGatherPer], b0[kGatherPer], b1[kGatherPer];
#pragma unroll
        for (int u = 0; u < kGatherPer; ++u) {
            const int e = cb + t + u * kGatherBlock;
            rr[u] = e < ce ? erec[e] : 0;
            wg[u] = e < ce ? wgt[e] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kGatherPer; ++u) {
            const int e = cb + t + u * kGatherBlock;
            b0[u] = e < ce ? rb0[rr[u]] : T(0);
            b1[u] = (e < ce && zg == 0) ? rb1[rr[u]] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kGatherPer; ++u) {
            const int i = t + u * kGatherBlock;
            p0s[i] = wg[u] * b0[u];
            p1s[i] = wg[u] * b1[u];
        }
        __syncthreads();
        const int lo = max(my0, cb), hi = min(my1, ce);
        for (int e = lo; e < hi; ++e) {
            s0 += p0s[e - cb];
            s1 += p1s[e - cb];
        }
        __syncthreads();   // the next chunk overwrites the products
    }
    if (t < mcount) {
        const long node = ga.node[zg][m0 + t];
        ga.out0[zg][node] += s0;
        if (zg == 0) ga.out1[node] += s1;
    }
}

// Transposed stencil map: for each node set, the (record, corner) pairs that
// touch each node, sorted by node, then record, then corner.
template <typename T>
int build_map(ibm_ctx* c) {
    AdjointMap& A = c->adj;
    const long nuv = c->rec[0].n, nw = c->rec[1].n, ntot = nuv + nw;
    const long plane = (long)c->g.nx * c->g.ny;
    const int nz = c->g.nz;
    std::vector<int32_t> base(ntot), sx(ntot), sy(ntot), ku(ntot), kw(ntot);
    std::vector<T> fx(ntot), fy(ntot), fzu(ntot), fzw(ntot);
    for (int kind = 0; kind < 2; ++kind) {
        const Records& R = c->rec[kind];
        if (R.n == 0) continue;
        const long o = kind ? nuv : 0;
        IBM_HIP(hipMemcpy(base.data() + o, R.base, 4 * R.n, hipMemcpyDeviceToHost));
        IBM_HIP(hipMemcpy(sx.data() + o, R.sx, 4 * R.n, hipMemcpyDeviceToHost));
        IBM_HIP(hipMemcpy(sy.data() + o, R.sy, 4 * R.n, hipMemcpyDeviceToHost));
        IBM_HIP(hipMemcpy(ku.data() + o, R.ku, 4 * R.n, hipMemcpyDeviceToHost));
        IBM_HIP(hipMemcpy(kw.data() + o, R.kw, 4 * R.n, hipMemcpyDeviceToHost));
        IBM_HIP(hipMemcpy(fx.data() + o, R.fx, sizeof(T) * R.n, hipMemcpyDeviceToHost));
        IBM_HIP(hipMemcpy(fy.data() + o, R.fy, sizeof(T) * R.n, hipMemcpyDeviceToHost));
        IBM_HIP(hipMemcpy(fzu.data() + o, R.fzu, sizeof(T) * R.n, hipMemcpyDeviceToHost));
        IBM_HIP(hipMemcpy(fzw.data() + o, R.fzw, sizeof(T) * R.n, hipMemcpyDeviceToHost));
    }
    for (int zg = 0; zg < 2; ++zg) {
        std::vector<uint64_t> key((size_t)ntot * 8);
        for (long rr = 0; rr < ntot; ++rr) {
            const int k0 = zg ? kw[rr] : ku[rr];
            const int k1 = std::min(k0 + 1, nz - 1);
            for (int cn = 0; cn < 8; ++cn) {
                const long node = (long)base[rr] + ((cn & 1) ? sx[rr] : 0) +
                                  ((cn & 2) ? sy[rr] : 0) + (long)((cn & 4) ? k1 : k0) * plane;
                key[(size_t)rr * 8 + cn] = ((uint64_t)node << 32) | ((uint64_t)rr << 3) | (uint64_t)cn;
            }
        }
        std::sort(key.begin(), key.end());
        std::vector<int32_t> node, off, erec(key.size());
        std::vector<T> wgt(key.size());
        for (size_t e = 0; e < key.size(); ++e) {
            const int32_t nd = (int32_t)(key[e] >> 32);
            if (node.empty() || node.back() != nd) {
                node.push_back(nd);
                off.push_back((int32_t)e);
            }
            const int32_t rr = (int32_t)((key[e] & 0xffffffffu) >> 3);
            const int cn = (int)(key[e] & 7u);
            erec[e] = rr;
            // the trilinear weight of this corner, in the storage type
            const T wz = zg ? fzw[rr] : fzu[rr];
            wgt[e] = ((cn & 1) ? fx[rr] : T(1) - fx[rr]) * ((cn & 2) ? fy[rr] : T(1) - fy[rr]) *
                     ((cn & 4) ? wz : T(1) - wz);
        }
        off.push_back((int32_t)key.size());
        A.m[zg] = (long)node.size();
        A.e[zg] = (long)key.size();
        const size_t nb = std::max<size_t>(node.size(), 1), eb = std::max<size_t>(key.size(), 1);
        IBM_HIP(hipMalloc(&A.node[zg], 4 * nb));
        IBM_HIP(hipMalloc(&A.off[zg], 4 * (nb + 1)));
        IBM_HIP(hipMalloc(&A.rec[zg], 4 * eb));
        IBM_HIP(hipMalloc(&A.wgt[zg], sizeof(T) * eb));
        if (!node.empty()) {
            IBM_HIP(hipMemcpy(A.node[zg], node.data(), 4 * node.size(), hipMemcpyHostToDevice));
            IBM_HIP(hipMemcpy(A.off[zg], off.data(), 4 * off.size(), hipMemcpyHostToDevice));
            IBM_HIP(hipMemcpy(A.rec[zg], erec.data(), 4 * erec.size(), hipMemcpyHostToDevice));
            IBM_HIP(hipMemcpy(A.wgt[zg], wgt.data(), sizeof(T) * wgt.size(), hipMemcpyHostToDevice));
        }
    }
    IBM_HIP(hipMalloc(&A.rbar, sizeof(T) * 3 * (size_t)std::max<long>(ntot, 1)));
    // band nodes in ascending order with their uv and w records
    std::vector<int32_t> qs[2];
    for (int kind = 0; kind < 2; ++kind) {
        qs[kind].resize(c->rec[kind].n);
        if (c->rec[kind].n)
            IBM_HIP(hipMemcpy(qs[kind].data(), c->rec[kind].q, 4 * c->rec[kind].n,
                              hipMemcpyDeviceToHost));
    }
    std::vector<int32_t> brec;
    brec.reserve(2 * (size_t)ntot);
    size_t iu = 0, iw = 0;
    while (iu < qs[0].size() || iw < qs[1].size()) {
        const int64_t qu = iu < qs[0].size() ? qs[0][iu] : INT64_MAX;
        const int64_t qw = iw < qs[1].size() ? qs[1][iw] : INT64_MAX;
        const int64_t q = std::min(qu, qw);
        brec.push_back(qu == q ? (int32_t)iu++ : -1);
        brec.push_back(qw == q ? (int32_t)iw++ : -1);
    }
    A.nb = (long)brec.size() / 2;
    IBM_HIP(hipMalloc(&A.brec, 4 * std::max<size_t>(brec.size(), 2)));
    if (!brec.empty())
        IBM_HIP(hipMemcpy(A.brec, brec.data(), 4 * brec.size(), hipMemcpyHostToDevice));
    A.built = true;
    return IBM_OK;
}

template <typename T>
int vjp_t(ibm_ctx* c, const T* u, const T* v, const T* w, double z0, const T* log_z0,
          const void* const g_tau[6], const void* const g_div[3], const void* const g_ustar[3],
          const double g_drag[3], T* gu, T* gv, T* gw, T* glz, hipStream_t s) {
    if (!c->adj.built) {
        IBM_HIP(hipStreamSynchronize(s));
        int rc = build_map<T>(c);
        if (rc) {
            free_adjoint(c);
            return rc;
        }
    }
    const long rows = (long)c->g.ny * c->g.nz;
    hipLaunchKernelGGL(k_vjp_dense<T>, dim3(nblk(c->n, 256)), dim3(256), 0, s,
                       (const T*)g_ustar[0], (const T*)g_ustar[1], (const T*)g_ustar[2], c->fmask,
                       c->g.nx, rows, c->wrow, gu, gv, gw, glz);
    const long nuv = c->rec[0].n, ntot = nuv + c->rec[1].n;
    BandArgs<T> a;
    a.u = u;
    a.v = v;
    a.w = w;
    a.log_z0 = log_z0;
    a.gt_mask = 0;
    for (int i = 0; i < 6; ++i) {
        a.g_tau[i] = g_tau ? (const T*)g_tau[i] : nullptr;
        if (a.g_tau[i]) a.gt_mask |= 1u << i;
    }
    for (int i = 0; i < 3; ++i) {
        a.g_div[i] = (const T*)g_div[i];
        a.gdrag[i] = g_drag[i];
    }
    a.fmask = c->fmask;
    a.nx = c->g.nx;
    a.ny = c->g.ny;
    a.nz = c->g.nz;
    a.wrow = c->wrow;
    a.plane = (long)c->g.nx * c->g.ny;
    a.dv = c->g.dx * c->g.dy * c->g.dz;
    a.cx = (T)(1.0 / (2.0 * c->g.dx));
    a.cy = (T)(1.0 / (2.0 * c->g.dy));
    a.cz = (T)(1.0 / c->g.dz);
    a.ln_scalar = log_z0 ? 0.0 : std::log(c->p.phi_c / z0);
    a.ln_phic = std::log(c->p.phi_c);
    a.kappa = c->p.kappa;
    a.dz = c->g.dz;
    a.mixed = c->precision == IBM_PREC_MIXED;
    a.rbar = (T*)c->adj.rbar;
    a.ntot = ntot;
    a.glz = glz;
    a.recs[0] = view<T>(c->rec[0]);
    a.recs[1] = view<T>(c->rec[1]);
    a.brec = c->adj.brec;
    a.nb = c->adj.nb;
    a.nuv = nuv;
    if (a.nb) {
        const dim3 gb(nblk(a.nb, 256));
        if (a.gt_mask) {
            for (int i = 0; i < 6; ++i)
                if (!a.g_tau[i]) a.g_tau[i] = a.g_div[0];   // read, never used
            if (log_z0)
                hipLaunchKernelGGL((k_vjp_band<T, true, true>), gb, dim3(256), 0, s, a);
            else
                hipLaunchKernelGGL((k_vjp_band<T, false, true>), gb, dim3(256), 0, s, a);
        } else if (log_z0) {
            hipLaunchKernelGGL((k_vjp_band<T, true, false>), gb, dim3(256), 0, s, a);
        } else {
            hipLaunchKernelGGL((k_vjp_band<T, false, false>), gb, dim3(256), 0, s, a);
        }
    }
    GatherArgs<T> ga;
    ga.ntot = ntot;
    ga.rbar = (const T*)c->adj.rbar;
    for (int zg = 0; zg < 2; ++zg) {
        ga.node[zg] = c->adj.node[zg];
        ga.off[zg] = c->adj.off[zg];
        ga.erec[zg] = c->adj.rec[zg];
        ga.wgt[zg] = (const T*)c->adj.wgt[zg];
        ga.m[zg] = c->adj.m[zg];
        ga.out0[zg] = zg ? gw : gu;
    }
    ga.out1 = gv;
    ga.nb0 = (int)nblk(ga.m[0], kGatherBlock);
    const unsigned gg = (unsigned)(ga.nb0 + nblk(ga.m[1], kGatherBlock));
    if (gg) hipLaunchKernelGGL(k_vjp_gather<T>, dim3(gg), dim3(kGatherBlock), 0, s, ga);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

}  // namespace

void free_adjoint(ibm_ctx* c) {
    AdjointMap& A = c->adj;
    for (int zg = 0; zg < 2; ++zg) {
        (void)hipFree(A.node[zg]);
        (void)hipFree(A.off[zg]);
        (void)hipFree(A.rec[zg]);
        (void)hipFree(A.wgt[zg]);
    }
    (void)hipFree(A.rbar);
    (void)hipFree(A.brec);
    A = AdjointMap();
}

int stage_vjp(ibm_ctx* c, const void* u, const void* v, const void* w, double z0,
              const void* log_z0, const void* const g_tau[6], const void* const g_div[3],
              const void* const g_ustar[3], const double g_drag[3], void* gu, void* gv, void* gw,
              void* glog_z0, hipStream_t s) {
    if (c->dtype == IBM_F64)
        return vjp_t<double>(c, (const double*)u, (const double*)v, (const double*)w, z0,
                             (const double*)log_z0, g_tau, g_div, g_ustar, g_drag, (double*)gu,
                             (double*)gv, (double*)gw, (double*)glog_z0, s);
    return vjp_t<float>(c, (const float*)u, (const float*)v, (const float*)w, z0,
                        (const float*)log_z0, g_tau, g_div, g_ustar, g_drag, (float*)gu,
                        (float*)gv, (float*)gw, (float*)glog_z0, s);
}

}  // namespace ibm
