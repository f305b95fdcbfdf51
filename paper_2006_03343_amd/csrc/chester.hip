// chester.hip -- Chester et al.'s original wall-modeled immersed boundary
// method, the comparison the paper improves on (§1; §3.3, closing
// paragraphs), on the GPU.  Its three steps:
//   1. the near-wall model in a fluid band 0 <= phi <= b of both node sets
//      (the original classifies the w and uv grids alike): the simplified
//      method's wall-stress device code (kernels.h, ws_block) on this band's
//      records, and zero stress at every node with phi < 0;
//   2. linear extrapolation into the solid band -b <= phi < 0: a solid-band
//      node samples its node set's stress components at the distances phi_c
//      and 2 phi_c from the surface along its normal and takes the straight
//      line through them at its own phi.  All values are formed into a
//      per-record buffer first (the samples may touch other solid-band nodes,
//      which still hold the 0 of step 1), then scattered;
//   3. red-black SOR of the 7-point Laplace equation over the interior
//      (phi < -b), every other node held fixed: one launch per colour and
//      sweep over compact lists of that colour's interior nodes.  With nx and
//      ny even no two nodes of one colour are neighbours, also across the
//      periodic seam, so each colour updates in place from the other's values.
// Set-up (once per geometry, after ibm_levelset_prepare): the class byte,
// ordered compaction of eight node lists (fluid band, solid band and the two
// colours of the interior, per node set), band and solid-band records
// (geom.h), and the segments holding a node with phi < 0.  The divergence,
// forcing and drag that follow are the simplified stage's (ibm_apply).
#include <algorithm>
#include <cmath>
#include <vector>

#include "geom.h"
#include "kernels.h"

namespace ibm {
namespace {

using namespace geom;

// list ids: fluid band uv, w; solid band uv, w; interior uv red, uv black,
// w red, w black
constexpr int kLists = 8;

__device__ inline int ch_class(double phi, double b) {
    return phi > b ? 0 : (phi >= 0.0 ? 1 : (phi >= -b ? 2 : 3));
}

template <typename T>
__global__ void k_ch_classify(const T* __restrict__ pu, const T* __restrict__ pw, long n,
                              double b, uint8_t* __restrict__ mask) {
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    mask[q] = (uint8_t)(ch_class((double)pu[q], b) | (ch_class((double)pw[q], b) << 2));
}

// List membership of node q (bit l set: node in list l).
__device__ inline unsigned ch_lists(uint8_t m, long q, int nx, int ny) {
    const int cu = m & 3, cw = (m >> 2) & 3;
    const long i = q % nx, j = (q / nx) % ny, k = q / ((long)nx * ny);
    const int colour = (int)((i + j + k) & 1);
    unsigned bits = 0;
    if (cu == 1) bits |= 1u << 0;
    if (cw == 1) bits |= 1u << 1;
    if (cu == 2) bits |= 1u << 2;
    if (cw == 2) bits |= 1u << 3;
    if (cu == 3) bits |= 1u << (4 + colour);
    if (cw == 3) bits |= 1u << (6 + colour);
    return bits;
}

// Per block of kNodesPerBlock nodes: the eight list counts, then the eight
// class counts (uv classes 0..3, w classes 0..3).
__global__ void __launch_bounds__(kCountBlock) k_ch_counts(const uint8_t* __restrict__ mask, long n,
                                                           int nx, int ny, int* __restrict__ bc) {
    __shared__ int lds[16][kCountBlock / 64];
    const long q0 = (long)blockIdx.x * kNodesPerBlock + (long)threadIdx.x * kItems;
    int c[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) c[i] = 0;
    for (int t = 0; t < kItems; ++t) {
        const long q = q0 + t;
        if (q >= n) break;
        const uint8_t m = mask[q];
        const unsigned bits = ch_lists(m, q, nx, ny);
#pragma unroll
        for (int l = 0; l < kLists; ++l) c[l] += (bits >> l) & 1u;
        c[8 + (m & 3)] += 1;
        c[12 + ((m >> 2) & 3)] += 1;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        int x = c[i];
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) x += __shfl_xor(x, s, 64);
        if (lane == 0) lds[i][w] = x;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        int s = 0;
        for (int i = 0; i < kCountBlock / 64; ++i) s += lds[threadIdx.x][i];
        bc[(long)blockIdx.x * 16 + threadIdx.x] = s;
    }
}

struct ListOut {
    int32_t* out[kLists];
};

// Ordered compaction: list l of block b starts at off[l * nb + b]; within the
// block, an exclusive scan per list keeps ascending linear index.
__global__ void __launch_bounds__(kCountBlock) k_ch_compact(const uint8_t* __restrict__ mask, long n,
                                                            int nx, int ny, long nb,
                                                            const long* __restrict__ off, ListOut lo) {
    __shared__ int lds[kCountBlock / 64];
    const long q0 = (long)blockIdx.x * kNodesPerBlock + (long)threadIdx.x * kItems;
    unsigned bits[kItems];
    int cnt[kLists];
#pragma unroll
    for (int l = 0; l < kLists; ++l) cnt[l] = 0;
    for (int t = 0; t < kItems; ++t) {
        const long q = q0 + t;
        bits[t] = q < n ? ch_lists(mask[q], q, nx, ny) : 0u;
#pragma unroll
        for (int l = 0; l < kLists; ++l) cnt[l] += (bits[t] >> l) & 1u;
    }
    for (int l = 0; l < kLists; ++l) {
        int tot;
        const int pre = block_exclusive_scan(cnt[l], lds, &tot);
        long o = off[(long)l * nb + blockIdx.x] + pre;
        for (int t = 0; t < kItems; ++t)
            if ((bits[t] >> l) & 1u) lo.out[l][o++] = (int32_t)(q0 + t);
    }
}

template <typename T, bool MIXED, bool HAS_LZ>
__global__ void __launch_bounds__(kBandBlock) k_ch_wall_stress(WSArgs<T> a) {
    ws_block<T, MIXED, HAS_LZ>(a, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_ch_finalize(const double* __restrict__ p, long nslots,
                                                     double* __restrict__ out) {
    finalize_slots(p, nslots, 4, 1u << 2, 1.0, out);
}

template <typename T>
struct ExtArgs {
    RecView<T> s1[2], s2[2];     // solid-band records: stencils at phi_c and 2 phi_c
    T* tau[6];
    T* ext;                      // [4 x uv records | 2 x w records]
    long plane;
    int nz;
    int nb_uv;                   // blocks of uv records
    T phic;
};

// Sample of one component at a record's stencil on the node set ``kind``.
template <typename T>
__device__ inline T ch_sample(const RecView<T>& R, long r, int kind, const T* f, long plane, int nz) {
    const long c00 = R.base[r], sx = R.sx[r], c01 = c00 + R.sy[r];
    const int k0 = kind == IBM_GRID_UV ? R.ku[r] : R.kw[r];
    const T fz = kind == IBM_GRID_UV ? R.fzu[r] : R.fzw[r];
    const long z0 = k0 * plane, z1 = min(k0 + 1, nz - 1) * plane;
    return trilerp_xpair<T>(f, c00, c01, sx, z0, z1, R.fx[r], R.fy[r], fz);
}

// Step 2, first half: one thread per solid-band record (uv blocks first).
template <typename T>
__global__ void __launch_bounds__(256) k_ch_extrapolate(ExtArgs<T> a) {
    const int kind = (int)blockIdx.x < a.nb_uv ? IBM_GRID_UV : IBM_GRID_W;
    const long r = (long)((int)blockIdx.x - (kind ? a.nb_uv : 0)) * blockDim.x + threadIdx.x;
    const RecView<T>& S1 = a.s1[kind];
    const RecView<T>& S2 = a.s2[kind];
    if (r >= S1.n) return;
    const T ph = S1.phi[r];
    const int c0 = kind == IBM_GRID_UV ? 0 : 4, nc = kind == IBM_GRID_UV ? 4 : 2;
    T* out = a.ext + (kind == IBM_GRID_UV ? 0 : 4 * a.s1[0].n);
    T v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (c >= nc) break;
        const T t1 = ch_sample<T>(S1, r, kind, a.tau[c0 + c], a.plane, a.nz);
        const T t2 = ch_sample<T>(S2, r, kind, a.tau[c0 + c], a.plane, a.nz);
        v[c] = t1 + (ph - a.phic) * (t2 - t1) / a.phic;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
        if (c < nc) out[(long)c * S1.n + r] = v[c];
}

// Step 2, second half: the extrapolated values into the stress fields.
template <typename T>
__global__ void __launch_bounds__(256) k_ch_scatter(ExtArgs<T> a) {
    const int kind = (int)blockIdx.x < a.nb_uv ? IBM_GRID_UV : IBM_GRID_W;
    const long r = (long)((int)blockIdx.x - (kind ? a.nb_uv : 0)) * blockDim.x + threadIdx.x;
    const RecView<T>& S1 = a.s1[kind];
    if (r >= S1.n) return;
    const long q = S1.q[r];
    const int c0 = kind == IBM_GRID_UV ? 0 : 4, nc = kind == IBM_GRID_UV ? 4 : 2;
    const T* in = a.ext + (kind == IBM_GRID_UV ? 0 : 4 * a.s1[0].n);
    for (int c = 0; c < nc; ++c) a.tau[c0 + c][q] = in[(long)c * S1.n + r];
}

template <typename T>
struct SorArgs {
    const int32_t* list[2];      // interior nodes of this colour, uv and w
    long n[2];
    int nb_uv;
    T* tau[6];
    int nx, ny, nz;
    long plane;
    T ax, ay, az, diag, omega, keep;   // 1/dx^2, 1/dy^2, 1/dz^2, 2 (sum), omega, 1 - omega
};

// Step 3: one half-sweep over the interior nodes of one colour (uv blocks
// first), each thread one node and every component of its node set.
template <typename T>
__global__ void __launch_bounds__(256) k_ch_sor(SorArgs<T> a) {
    const int kind = (int)blockIdx.x < a.nb_uv ? IBM_GRID_UV : IBM_GRID_W;
    const long r = (long)((int)blockIdx.x - (kind ? a.nb_uv : 0)) * blockDim.x + threadIdx.x;
    if (r >= a.n[kind]) return;
    const long q = a.list[kind][r];
    const int nx = a.nx, ny = a.ny;
    const int i = (int)(q % nx);
    const long jk = q / nx;
    const int j = (int)(jk % ny);
    const int k = (int)(jk / ny);
    const long xm = q + (i == 0 ? nx - 1 : -1), xp = q + (i == nx - 1 ? 1 - nx : 1);
    const long row = (long)nx;
    const long ym = q + (j == 0 ? (long)(ny - 1) * row : -row);
    const long yp = q + (j == ny - 1 ? (long)(1 - ny) * row : row);
    const bool hasd = k > 0, hasu = k < a.nz - 1;
    const int c0 = kind == IBM_GRID_UV ? 0 : 4, nc = kind == IBM_GRID_UV ? 4 : 2;
    T nv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (c >= nc) break;
        const T* __restrict__ f = a.tau[c0 + c];
        const T d = hasd ? f[q - a.plane] : T(0);
        const T u = hasu ? f[q + a.plane] : T(0);
        const T s = a.ax * (f[xp] + f[xm]) + a.ay * (f[yp] + f[ym]) + a.az * (u + d);
        nv[c] = a.keep * f[q] + a.omega * s / a.diag;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
        if (c < nc) a.tau[c0 + c][q] = nv[c];
}

inline unsigned nblk_(long n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename T>
int chester_prepare_t(ibm_ctx* c, const T* pu, const T* pw, hipStream_t s) {
    ChesterGeom& G = c->ch;
    const long n = c->n;
    const int nx = c->g.nx, ny = c->g.ny, nz = c->g.nz;
    const double b = c->p.band_width;
    IBM_HIP(hipMalloc(&G.mask, (size_t)n));
    hipLaunchKernelGGL(k_ch_classify<T>, dim3(nblk_(n, 256)), dim3(256), 0, s, pu, pw, n, b, G.mask);
    const long nb = (n + kNodesPerBlock - 1) / kNodesPerBlock;
    int* bc = nullptr;
    IBM_HIP(hipMalloc(&bc, sizeof(int) * 16 * (size_t)nb));
    hipLaunchKernelGGL(k_ch_counts, dim3((unsigned)nb), dim3(kCountBlock), 0, s, G.mask, n, nx, ny,
                       bc);
    IBM_HIP(hipGetLastError());
    std::vector<int> hbc(16 * (size_t)nb);
    IBM_HIP(hipMemcpyAsync(hbc.data(), bc, sizeof(int) * 16 * (size_t)nb, hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    (void)hipFree(bc);
    std::vector<long> off((size_t)kLists * nb);
    long tot[kLists] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < 8; ++i) G.counts[i] = 0;
    for (long k = 0; k < nb; ++k) {
        for (int l = 0; l < kLists; ++l) {
            off[(size_t)l * nb + k] = tot[l];
            tot[l] += hbc[16 * k + l];
        }
        for (int i = 0; i < 8; ++i) G.counts[i] += hbc[16 * k + 8 + i];
    }
    // records of the fluid band (0, 1) and solid band (2, 3); interior lists
    int rc;
    for (int kind = 0; kind < 2; ++kind) {
        if ((rc = alloc_records(G.band[kind], tot[kind], sizeof(T)))) return rc;
        if ((rc = alloc_records(G.sb1[kind], tot[2 + kind], sizeof(T)))) return rc;
        if ((rc = alloc_records(G.sb2[kind], tot[2 + kind], sizeof(T)))) return rc;
    }
    long nin = 0;
    for (int l = 4; l < kLists; ++l) nin += tot[l];
    IBM_HIP(hipMalloc(&G.lists, sizeof(int32_t) * (size_t)std::max<long>(nin, 1)));
    ListOut lo;
    lo.out[0] = G.band[0].q;
    lo.out[1] = G.band[1].q;
    lo.out[2] = G.sb1[0].q;
    lo.out[3] = G.sb1[1].q;
    int32_t* p = (int32_t*)G.lists;
    for (int l = 4; l < kLists; ++l) {
        const int kind = (l - 4) / 2, colour = (l - 4) % 2;
        G.inner[kind][colour] = p;
        G.ninner[kind][colour] = tot[l];
        lo.out[l] = p;
        p += tot[l];
    }
    long* doff = nullptr;
    IBM_HIP(hipMalloc(&doff, sizeof(long) * off.size()));
    IBM_HIP(hipMemcpyAsync(doff, off.data(), sizeof(long) * off.size(), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ch_compact, dim3((unsigned)nb), dim3(kCountBlock), 0, s, G.mask, n, nx, ny,
                       nb, doff, lo);
    for (int kind = 0; kind < 2; ++kind)
        if (G.sb1[kind].n)
            IBM_HIP(hipMemcpyAsync(G.sb2[kind].q, G.sb1[kind].q, sizeof(int32_t) * G.sb1[kind].n,
                                   hipMemcpyDeviceToDevice, s));
    const bool mixed = c->precision == IBM_PREC_MIXED;
    auto build = [&](Records& R, int kind, double dist) {
        if (R.n == 0) return;
        RecOut o{R.q, R.base, R.sx, R.sy, R.ku, R.kw, R.nrm[0], R.nrm[1], R.nrm[2], R.phi,
                 R.fx, R.fy, R.fzu, R.fzw};
        GeomArgs ga{nx, ny, nz, c->g.dx, c->g.dy, c->g.dz, dist};
        const T* ph = kind == 0 ? pu : pw;
        if (mixed)
            hipLaunchKernelGGL((k_records<T, true>), dim3(nblk_(R.n, 256)), dim3(256), 0, s, ph,
                               kind, R.n, o, ga);
        else
            hipLaunchKernelGGL((k_records<T, false>), dim3(nblk_(R.n, 256)), dim3(256), 0, s, ph,
                               kind, R.n, o, ga);
    };
    for (int kind = 0; kind < 2; ++kind) {
        build(G.band[kind], kind, c->p.phi_c);
        build(G.sb1[kind], kind, c->p.phi_c);
        build(G.sb2[kind], kind, 2.0 * c->p.phi_c);
    }
    IBM_HIP(hipMalloc(&G.ext, sizeof(T) * (size_t)std::max<long>(4 * tot[2] + 2 * tot[3], 1)));
    const long nbb = std::max<long>(1, (long)nblk_(tot[0], kBandBlock) + (long)nblk_(tot[1], kBandBlock));
    IBM_HIP(hipMalloc(&G.partials, sizeof(double) * 4 * (size_t)nbb));
    // segments holding a node with phi < 0 (class 2 or 3) on either set
    const long nseg = (n + kSeg - 1) / kSeg;
    uint8_t* dflags = nullptr;
    IBM_HIP(hipMalloc(&dflags, (size_t)nseg));
    hipLaunchKernelGGL(k_seg_flags, dim3((unsigned)nseg), dim3(256), 0, s, G.mask, n, dflags);
    IBM_HIP(hipGetLastError());
    std::vector<uint8_t> hf(nseg);
    IBM_HIP(hipMemcpyAsync(hf.data(), dflags, (size_t)nseg, hipMemcpyDeviceToHost, s));
    IBM_HIP(hipStreamSynchronize(s));
    (void)hipFree(dflags);
    (void)hipFree(doff);
    std::vector<Seg> zs;
    for (long i = 0; i < nseg; ++i)
        if (hf[i] & 3)
            zs.push_back(Seg{(int32_t)(i * kSeg), (int32_t)std::min<long>(kSeg, n - i * kSeg),
                             hf[i] & 3, 0});
    G.nzsegs = (long)zs.size();
    IBM_HIP(hipMalloc(&G.zsegs, sizeof(Seg) * std::max<size_t>(zs.size(), 1)));
    if (!zs.empty())
        IBM_HIP(hipMemcpy(G.zsegs, zs.data(), sizeof(Seg) * zs.size(), hipMemcpyHostToDevice));
    return IBM_OK;
}

template <typename T>
int chester_wall_stress_t(ibm_ctx* c, const T* u, const T* v, const T* w, double z0,
                          const T* log_z0, void* const tau[6], double omega, int iterations,
                          double* stats, hipStream_t s) {
    const ChesterGeom& G = c->ch;
    const long plane = (long)c->g.nx * c->g.ny;
    // step 1: the simplified method's wall-stress blocks on the fluid band
    WSArgs<T> a;
    a.rec[0] = view<T>(G.band[0]);
    a.rec[1] = view<T>(G.band[1]);
    a.u = u;
    a.v = v;
    a.w = w;
    a.log_z0 = log_z0;
    for (int i = 0; i < 6; ++i) a.tau[i] = (T*)tau[i];
    a.zsegs = G.zsegs;
    a.mask = G.mask;
    a.nx = c->g.nx;
    a.ny = c->g.ny;
    a.nz = c->g.nz;
    a.plane = plane;
    a.nb_uv = (int)nblk_(G.band[0].n, kBandBlock);
    a.nb_band = (int)std::max<long>(1, (long)a.nb_uv + (long)nblk_(G.band[1].n, kBandBlock));
    a.ln_scalar = log_z0 ? 0.0 : std::log(c->p.phi_c / z0);
    a.ln_phic = std::log(c->p.phi_c);
    a.kappa = c->p.kappa;
    a.dz = c->g.dz;
    a.partials = G.partials;
    a.stats = stats;
    const unsigned grid = (unsigned)(a.nb_band + G.nzsegs);
    const bool mixed = c->precision == IBM_PREC_MIXED;
    if (mixed && log_z0)
        hipLaunchKernelGGL((k_ch_wall_stress<T, true, true>), dim3(grid), dim3(kBandBlock), 0, s, a);
    else if (mixed)
        hipLaunchKernelGGL((k_ch_wall_stress<T, true, false>), dim3(grid), dim3(kBandBlock), 0, s, a);
    else if (log_z0)
        hipLaunchKernelGGL((k_ch_wall_stress<T, false, true>), dim3(grid), dim3(kBandBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_ch_wall_stress<T, false, false>), dim3(grid), dim3(kBandBlock), 0, s, a);
    if (stats)
        hipLaunchKernelGGL(k_ch_finalize, dim3(1), dim3(256), 0, s, (const double*)G.partials,
                           (long)a.nb_band, stats);
    // step 2: extrapolation into the solid band
    ExtArgs<T> e;
    for (int k = 0; k < 2; ++k) {
        e.s1[k] = view<T>(G.sb1[k]);
        e.s2[k] = view<T>(G.sb2[k]);
    }
    for (int i = 0; i < 6; ++i) e.tau[i] = (T*)tau[i];
    e.ext = (T*)G.ext;
    e.plane = plane;
    e.nz = c->g.nz;
    e.nb_uv = (int)nblk_(G.sb1[0].n, 256);
    e.phic = (T)c->p.phi_c;
    const unsigned ge = (unsigned)(e.nb_uv + nblk_(G.sb1[1].n, 256));
    if (ge) {
        hipLaunchKernelGGL(k_ch_extrapolate<T>, dim3(ge), dim3(256), 0, s, e);
        hipLaunchKernelGGL(k_ch_scatter<T>, dim3(ge), dim3(256), 0, s, e);
    }
    // step 3: red-black SOR over the interior
    SorArgs<T> sa[2];
    for (int colour = 0; colour < 2; ++colour) {
        SorArgs<T>& q = sa[colour];
        for (int k = 0; k < 2; ++k) {
            q.list[k] = G.inner[k][colour];
            q.n[k] = G.ninner[k][colour];
        }
        q.nb_uv = (int)nblk_(q.n[0], 256);
        for (int i = 0; i < 6; ++i) q.tau[i] = (T*)tau[i];
        q.nx = c->g.nx;
        q.ny = c->g.ny;
        q.nz = c->g.nz;
        q.plane = plane;
        const double ax = 1.0 / (c->g.dx * c->g.dx), ay = 1.0 / (c->g.dy * c->g.dy),
                     az = 1.0 / (c->g.dz * c->g.dz);
        q.ax = (T)ax;
        q.ay = (T)ay;
        q.az = (T)az;
        q.diag = (T)(2.0 * (ax + ay + az));
        q.omega = (T)omega;
        q.keep = (T)(1.0 - omega);
    }
    const unsigned gs[2] = {(unsigned)(sa[0].nb_uv + nblk_(sa[0].n[1], 256)),
                            (unsigned)(sa[1].nb_uv + nblk_(sa[1].n[1], 256))};
    for (int it = 0; it < iterations; ++it)
        for (int colour = 0; colour < 2; ++colour)
            if (gs[colour])
                hipLaunchKernelGGL(k_ch_sor<T>, dim3(gs[colour]), dim3(256), 0, s, sa[colour]);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

}  // namespace

void free_chester(ibm_ctx* c) {
    ChesterGeom& G = c->ch;
    (void)hipFree(G.mask);
    for (int k = 0; k < 2; ++k) {
        (void)hipFree(G.band[k].buf);
        (void)hipFree(G.sb1[k].buf);
        (void)hipFree(G.sb2[k].buf);
    }
    (void)hipFree(G.lists);
    (void)hipFree(G.ext);
    (void)hipFree(G.zsegs);
    (void)hipFree(G.partials);
    G = ChesterGeom();
}

int chester_prepare(ibm_ctx* c, const void* phi_uv, const void* phi_w, hipStream_t s) {
    free_chester(c);
    const int rc = c->dtype == IBM_F64
                       ? chester_prepare_t<double>(c, (const double*)phi_uv, (const double*)phi_w, s)
                       : chester_prepare_t<float>(c, (const float*)phi_uv, (const float*)phi_w, s);
    if (rc != IBM_OK) {
        free_chester(c);
        return rc;
    }
    c->ch.built = true;
    return IBM_OK;
}

int launch_chester_wall_stress(ibm_ctx* c, const void* u, const void* v, const void* w,
                               double z0, const void* log_z0, void* const tau[6], double omega,
                               int iterations, double* stats, hipStream_t s) {
    if (c->dtype == IBM_F64)
        return chester_wall_stress_t<double>(c, (const double*)u, (const double*)v,
                                             (const double*)w, z0, (const double*)log_z0, tau,
                                             omega, iterations, stats, s);
    return chester_wall_stress_t<float>(c, (const float*)u, (const float*)v, (const float*)w, z0,
                                        (const float*)log_z0, tau, omega, iterations, stats, s);
}

}  // namespace ibm
