// spectral.hip -- the stress divergence with the paper's own pseudo-spectral
// horizontal derivatives (§2.4, eq. dudx) instead of central differences:
//   d/dx A = sum over wavenumbers of i k A_hat exp(i k x), periodic in x and
//   y, the Nyquist mode of an even node count without derivative; the
//   vertical staggered differences (eqs. dudz, dwdz), the forcing (eq.
//   u-*-IBM) and the drag are those of the dense pass.
//
// Two launches (and the drag finalize):
//   k_dx   a thread team per pair of rows (r, r+1) holds three complex
//          sequences in registers: tau_xx + i tau_xy of each row and
//          tau_xz of row r + i tau_xz of row r+1 (the derivative is a real
//          operator, so the real and imaginary parts stay apart); forward
//          transform, product with i k / nx with the Nyquist mode dropped
//          (explicitly: with two fields packed its term would leak into the
//          other field), inverse transform; writes div_x = d/dx tau_xx,
//          div_y = d/dx tau_xy, div_z = d/dx tau_xz; the blocks after the row
//          blocks force the forcing segments;
//   k_dy   the same along y with one divergence component per block: a team
//          per pair of columns (c, c+1) of one plane transforms tau_xy,
//          tau_yy or tau_yz of the two columns as one sequence, adds d/dy of
//          it and the staggered vertical difference of the component's third
//          term (d/dz tau_xz, tau_yz on uv nodes, d/dz tau_zz on w nodes, zero
//          padded), loaded with the divergence it updates; with the final
//          divergence component in hand it leaves its drag partial over the
//          fluid nodes, summed in slot order by k_spec_finalize.  The three
//          components of a plane's column group are consecutive blocks of one
//          XCD, so the lines they share (tau_yz, the flags) meet in its L2.
// The y pass with all three sequences in one team needed about 200 registers
// (two waves per SIMD) and ran at 3.7 TB/s; with one it holds 68 (seven waves)
// and, in 512-thread blocks whose row segments are whole cache lines, runs at
// 5.4 TB/s on the bytes it moves.  The x pass, whose three sequences are one
// stress row each, is faster with all three in one team (225 against 275 us
// on the 512 x 256 x 256 hill): split, its blocks each stage the twiddles and
// run two transforms for a third of the data.
// Transforms: fft.h (register-resident Stockham passes of radix 8, thread
// teams of n / 8).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "fft.h"
#include "kernels.h"

namespace ibm {
namespace {

template <typename T>
struct SpecArgs {
    const T* tau[6];
    T* div[3];
    const Cx<T>* twx;
    const Cx<T>* twy;
    int nx, ny, nz, logx, logy;
    long rows;               // ny * nz
    long plane;              // nx * ny
    T kx, ky;                // 2 pi / Lx, 2 pi / Ly
    T cz;                    // 1 / dz
};

// i k_m X_m / n for every slot (the Nyquist mode gets k = 0).
template <typename T, int S>
__device__ inline void derivative(Cx<T> (&v)[S][8], const Team& tm, int n, T two_pi_over_len) {
    const T inv_n = T(1) / T(n);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const T k = two_pi_over_len * T(mode_number(tm.elem(u) & (n - 1), n)) * inv_n;
#pragma unroll
        for (int s = 0; s < S; ++s) v[s][u] = Cx<T>{-(k * v[s][u].im), k * v[s][u].re};
    }
}

template <typename T>
struct alignas(2 * sizeof(T)) Two {
    T x, y;
};

// Staggered vertical difference of tau component c at node q of plane k:
// on uv nodes (up) (tau[q + plane] - tau[q]) / dz, on w nodes (tau[q] -
// tau[q - plane]) / dz, zero beyond the top and bottom planes.
template <typename T>
__device__ inline T zdiff(const SpecArgs<T>& a, int c, long q, int k, bool up) {
    const T* t = a.tau[c];
    if (up) return ((k + 1 < a.nz ? t[q + a.plane] : T(0)) - t[q]) * a.cz;
    return (t[q] - (k > 0 ? t[q - a.plane] : T(0))) * a.cz;
}

// The same for the two nodes q, q + 1 (q even, fields 8-byte aligned).
template <typename T>
__device__ inline Two<T> zdiff2(const SpecArgs<T>& a, int c, long q, int k, bool up) {
    const T* t = a.tau[c];
    const Two<T> z{T(0), T(0)};
    const Two<T> here = *reinterpret_cast<const Two<T>*>(t + q);
    if (up) {
        const Two<T> nb = k + 1 < a.nz ? *reinterpret_cast<const Two<T>*>(t + q + a.plane) : z;
        return Two<T>{(nb.x - here.x) * a.cz, (nb.y - here.y) * a.cz};
    }
    const Two<T> nb = k > 0 ? *reinterpret_cast<const Two<T>*>(t + q - a.plane) : z;
    return Two<T>{(here.x - nb.x) * a.cz, (here.y - nb.y) * a.cz};
}

// Stress component differenced along y for divergence component c.
__device__ inline int yfield(int c) { return c == 0 ? 3 : c == 1 ? 1 : 5; }   // xy, yy, yz

// Sequences a team transforms at once: all three in float; one after another
// in double, whose registers would spill otherwise.
template <typename T>
constexpr int kSeqAtOnce = sizeof(T) == 4 ? 3 : 1;

// A team of P = max(1, nx / 8) consecutive threads per pair of rows (r, r+1);
// sequence 0 = tau_xx + i tau_xy of row r, 1 = the same of row r+1, 2 =
// tau_xz of row r + i tau_xz of row r+1.
template <typename T, bool ALL>
__global__ void __launch_bounds__(256) k_dx(SpecArgs<T> a, ApplyArgs<T> z, unsigned nrowblocks) {
    if (blockIdx.x >= nrowblocks) {
        // forcing: quarters of the forcing segments
        constexpr int kPiece = kSeg / 4;
        for (long it = blockIdx.x - nrowblocks; it < 4 * z.nfsegs; it += z.nfblocks) {
            const Seg sg = z.fsegs[it >> 2];
            const int off = (int)(it & 3) * kPiece;
            if (off < sg.len)
                force_seg<T>(z, Seg{sg.q + off, min(kPiece, sg.len - off), 0, 0}, threadIdx.x,
                             blockDim.x);
        }
        return;
    }
    constexpr int G = kSeqAtOnce<T>;
    extern __shared__ unsigned char lds_raw[];
    Cx<T>* xl = reinterpret_cast<Cx<T>*>(lds_raw);
    const int n = a.nx, logn = a.logx;
    const int P = n >= 8 ? n >> 3 : 1, ns = n >= 8 ? 8 : n;
    const int teams = (int)blockDim.x / P;
    Cx<T>* tw = xl + team_lds_elems(blockDim.x) * (ALL ? G : 1);
    stage_twiddles(tw, a.twx, n);
    const int team = (int)threadIdx.x / P;
    const Team tm = make_team(logn, (int)threadIdx.x - team * P, team, teams, false);
    const long r0 = 2 * ((long)blockIdx.x * teams + team);
    const bool in[2] = {r0 < a.rows, r0 + 1 < a.rows};
    for (int s0 = 0; s0 < 3; s0 += G) {
        Cx<T> v[G][8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const long o = r0 * n + tm.elem(u);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int sq = s0 + g;
                v[g][u] = Cx<T>{T(0), T(0)};
                if (u >= ns) continue;
                if (sq < 2) {
                    if (in[sq]) v[g][u] = Cx<T>{a.tau[0][o + sq * n], a.tau[3][o + sq * n]};
                } else {
                    if (in[0]) v[g][u].re = a.tau[4][o];
                    if (in[1]) v[g][u].im = a.tau[4][o + n];
                }
            }
        }
        __syncthreads();   // twiddles staged; the previous group's exchanges done
        team_fft<T, G, ALL>(v, tm, xl, tw);
        derivative<T, G>(v, tm, n, a.kx);
        team_ifft<T, G, ALL>(v, tm, xl, tw);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (u >= ns) continue;
            const long o = r0 * n + tm.elem(u);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int sq = s0 + g;
                if (sq < 2) {
                    if (in[sq]) {
                        a.div[0][o + sq * n] = v[g][u].re;
                        a.div[1][o + sq * n] = v[g][u].im;
                    }
                } else {
                    if (in[0]) a.div[2][o] = v[g][u].re;
                    if (in[1]) a.div[2][o + n] = v[g][u].im;
                }
            }
        }
    }
}

// Logical block lb (XCD-aware): component c = lb % 3 of column group lb / 3
// = (plane k, group gi); a team per pair of columns (c0, c0+1) of plane k,
// the teams of a block interleaved across lanes (lane = j * teams + team) so
// a row's columns are read together; sequence tau(c0) + i tau(c0+1) along y.
// PAIR (nx even, fields aligned to two elements): the two columns of a field
// move as one access.
// Threads per y-pass block: in float 16 teams of a 256-point transform, so a
// block's row segment is a whole 128-byte line of column pairs; in double 8
// teams already move two lines, and their exchanges fill 64 KiB of LDS at the
// longest transform.
template <typename T>
constexpr int kDyThreads = sizeof(T) == 4 ? 512 : 256;

template <typename T, bool PAIR, typename Acc>
__global__ void __launch_bounds__(kDyThreads<T>) k_dy(SpecArgs<T> a, ApplyArgs<T> z) {
    extern __shared__ unsigned char lds_raw[];
    Cx<T>* xl = reinterpret_cast<Cx<T>*>(lds_raw);
    const int n = a.ny, logn = a.logy;
    const int P = n >= 8 ? n >> 3 : 1, ns = n >= 8 ? 8 : n;
    const int teams = (int)blockDim.x / P;
    const int groups = (a.nx + 2 * teams - 1) / (2 * teams);
    const int lb = xcd_block(3 * groups * a.nz);
    if (lb < 0) return;                                   // the whole block
    Cx<T>* tw = xl + team_lds_elems(blockDim.x);
    stage_twiddles(tw, a.twy, n);
    const int comp = lb % 3;
    const int rest = lb / 3;
    const int k = rest / groups;
    const int gi = rest - k * groups;
    const int team = (int)threadIdx.x % teams;
    const Team tm = make_team(logn, (int)threadIdx.x / teams, team, teams, true);
    const int c0 = 2 * (gi * teams + team);
    const bool in0 = c0 < a.nx, in1 = c0 + 1 < a.nx;
    const long pk = (long)k * a.ny * a.nx;
    const T* __restrict__ f = a.tau[yfield(comp)];
    const int zc = comp == 0 ? 4 : comp == 1 ? 5 : 2;    // tau_xz, tau_yz up; tau_zz down
    const bool up = comp < 2;
    const uint32_t fbit = comp < 2 ? 1u : 2u;            // forced uv node / forced w node
    T* __restrict__ d = a.div[comp];
    Cx<T> v[1][8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        v[0][u] = Cx<T>{T(0), T(0)};
        if (u >= ns || !in0) continue;
        const long q = pk + (long)tm.elem(u) * a.nx + c0;
        if constexpr (PAIR) {
            const Two<T> t = *reinterpret_cast<const Two<T>*>(f + q);
            v[0][u] = Cx<T>{t.x, t.y};
        } else {
            v[0][u] = Cx<T>{f[q], in1 ? f[q + 1] : T(0)};
        }
    }
    __syncthreads();
    team_fft<T, 1>(v, tm, xl, tw);
    derivative<T, 1>(v, tm, n, a.ky);
    team_ifft<T, 1>(v, tm, xl, tw);
    Acc acc = Acc(0);                                     // drag partial over the fluid nodes
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        if (u >= ns || !in0) continue;
        const int row = tm.elem(u);
        const long q = pk + (long)row * a.nx + c0;
        // forcing flags of columns c0, c0 + 1 (one word: c0 is even)
        const uint32_t fw = z.fmask[((long)k * a.ny + row) * z.wrow + (c0 >> 4)] >> (2 * (c0 & 15));
        if constexpr (PAIR) {
            Two<T>* dp = reinterpret_cast<Two<T>*>(d + q);
            const Two<T> o = *dp;
            // the staggered vertical difference, loaded with the divergence
            const Two<T> zd = zdiff2(a, zc, q, k, up);
            const Two<T> r{o.x + v[0][u].re + zd.x, o.y + v[0][u].im + zd.y};
            *dp = r;
            if (!(fw & fbit)) acc += (Acc)r.x;
            if (in1 && !((fw >> 2) & fbit)) acc += (Acc)r.y;
        } else {
            const T r0v = d[q] + v[0][u].re + zdiff(a, zc, q, k, up);
            d[q] = r0v;
            if (!(fw & fbit)) acc += (Acc)r0v;
            if (in1) {
                const T r1v = d[q + 1] + v[0][u].im + zdiff(a, zc, q + 1, k, up);
                d[q + 1] = r1v;
                if (!((fw >> 2) & fbit)) acc += (Acc)r1v;
            }
        }
    }
    if (!z.drag) return;
    __shared__ double red[kDyThreads<T> / 64];
    const double ws = wave_sum((double)acc);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = ws;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += red[w];
        z.partials[3L * rest + comp] = r;     // slot of (plane, group), component comp
    }
}

__global__ void __launch_bounds__(256) k_spec_finalize(const double* __restrict__ p, long nslots,
                                                       double scale, double* __restrict__ out) {
    finalize_slots(p, nslots, 3, 0u, scale, out);
}

void free_spectral_tables(ibm_ctx* c) {
    (void)hipFree(c->spec.twx);
    (void)hipFree(c->spec.twy);
    c->spec.twx = c->spec.twy = nullptr;
}

int ilog2_exact(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return (1 << l) == n ? l : -1;
}

template <typename T>
int twiddles(ibm_ctx* c, int n, void** dst) {
    std::vector<Cx<T>> t(n);
    for (int i = 0; i < n; ++i) {
        const double ang = -2.0 * M_PI * (double)i / (double)n;
        t[i] = Cx<T>{(T)std::cos(ang), (T)std::sin(ang)};
    }
    IBM_HIP(hipMalloc(dst, sizeof(Cx<T>) * t.size()));
    IBM_HIP(hipMemcpy(*dst, t.data(), sizeof(Cx<T>) * t.size(), hipMemcpyHostToDevice));
    return IBM_OK;
}

template <typename T>
int spectral_t(ibm_ctx* c, const void* const tau[6], void* const ustar[3],
               const void* const gradp[3], double dt, void* const div[3], double* drag,
               hipStream_t s) {
    const int nx = c->g.nx, ny = c->g.ny, nz = c->g.nz;
    const int lx = ilog2_exact(nx), ly = ilog2_exact(ny);
    int rc = spectral_check(c);
    if (rc) return rc;
    if ((rc = ensure_twiddles(c))) return rc;
    SpecArgs<T> a;
    for (int i = 0; i < 6; ++i) a.tau[i] = (const T*)tau[i];
    for (int i = 0; i < 3; ++i) a.div[i] = (T*)div[i];
    a.twx = (const Cx<T>*)c->spec.twx;
    a.twy = (const Cx<T>*)c->spec.twy;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.logx = lx;
    a.logy = ly;
    a.rows = (long)ny * nz;
    a.plane = (long)nx * ny;
    a.kx = (T)(2.0 * M_PI / (nx * c->g.dx));
    a.ky = (T)(2.0 * M_PI / (ny * c->g.dy));
    a.cz = (T)(1.0 / c->g.dz);
    ApplyArgs<T> z = make_apply_args<T>(c, c->cfg, tau, ustar, gradp, dt, div, drag);
    const int ty = kDyThreads<T> / (ny >= 8 ? ny / 8 : 1);
    const int groups = (nx + 2 * ty - 1) / (2 * ty);
    const long nsl = (long)groups * nz;                     // drag slots: one per column group
    const long nyb = 3 * nsl;                               // y-pass blocks: three per group
    if (c->ap_cap < 3L * nsl) return fail(IBM_E_STATE, "apply_spectral: reduction slots not sized");
    z.partials = c->ap_partials;
    z.nfblocks = (int)std::min<long>((4 * c->nfsegs + 7) / 8 * 8, 2048);
    const int tx = 256 / (nx >= 8 ? nx / 8 : 1);            // teams per block
    const long pairs = (a.rows + 1) / 2;
    const unsigned nrb = (unsigned)((pairs + tx - 1) / tx);
    // one sequence's exchange space: exchanging all three at once measured
    // slower here (more registers, fewer waves)
    hipLaunchKernelGGL((k_dx<T, false>), dim3(nrb + (unsigned)z.nfblocks), dim3(256),
                       spectral_lds_bytes(c, nx, 1), s, a, z, nrb);
    bool aligned = nx % 2 == 0;
    for (int i = 0; i < 6; ++i) aligned = aligned && (uintptr_t)tau[i] % (2 * sizeof(T)) == 0;
    for (int i = 0; i < 3; ++i) aligned = aligned && (uintptr_t)div[i] % (2 * sizeof(T)) == 0;
    const bool wide = c->precision == IBM_PREC_MIXED || sizeof(T) == 8;   // drag in double
    const dim3 gdy((unsigned)(8 * ((nyb + 7) / 8)));     // logical blocks dealt per XCD
    const size_t lds_y = spectral_lds_bytes(c, ny, 1, kDyThreads<T>);
    if (aligned && wide)
        hipLaunchKernelGGL((k_dy<T, true, double>), gdy, dim3(kDyThreads<T>), lds_y, s, a, z);
    else if (aligned)
        hipLaunchKernelGGL((k_dy<T, true, T>), gdy, dim3(kDyThreads<T>), lds_y, s, a, z);
    else if (wide)
        hipLaunchKernelGGL((k_dy<T, false, double>), gdy, dim3(kDyThreads<T>), lds_y, s, a, z);
    else
        hipLaunchKernelGGL((k_dy<T, false, T>), gdy, dim3(kDyThreads<T>), lds_y, s, a, z);
    if (drag)
        hipLaunchKernelGGL(k_spec_finalize, dim3(1), dim3(256), 0, s, (const double*)z.partials,
                           nsl, z.dv, drag);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

}  // namespace

int ensure_twiddles(ibm_ctx* c) {
    if (c->spec.twx && c->spec.twy) return IBM_OK;
    void *tx = nullptr, *ty = nullptr;
    int rc = c->dtype == IBM_F64 ? twiddles<double>(c, c->g.nx, &tx) : twiddles<float>(c, c->g.nx, &tx);
    if (!rc)
        rc = c->dtype == IBM_F64 ? twiddles<double>(c, c->g.ny, &ty) : twiddles<float>(c, c->g.ny, &ty);
    if (rc) {
        (void)hipFree(tx);
        (void)hipFree(ty);
        return rc;
    }
    free_spectral_tables(c);
    c->spec.twx = tx;
    c->spec.twy = ty;
    return IBM_OK;
}

namespace {

// The longest transform of the storage type: a team of n / 8 threads within a
// 256-thread block; LDS for the teams' exchanges and the twiddle table within
// 64 KiB.
int max_length(const ibm_ctx* c) { return c->dtype == IBM_F64 ? 1024 : 2048; }

// Whether the transforms take this grid (spectral_check without the message).
bool spectral_fits(const ibm_ctx* c) {
    return ilog2_exact(c->g.nx) >= 0 && ilog2_exact(c->g.ny) >= 0 && c->g.nx <= max_length(c) &&
           c->g.ny <= max_length(c);
}

}  // namespace

int spectral_check(const ibm_ctx* c) {
    const int nx = c->g.nx, ny = c->g.ny;
    if (ilog2_exact(nx) < 0 || ilog2_exact(ny) < 0)
        return fail(IBM_E_UNSUPPORTED, "spectral transforms: nx and ny must be powers of two (%d, %d)",
                    nx, ny);
    const int nmax = max_length(c);
    if (nx > nmax || ny > nmax)
        return fail(IBM_E_UNSUPPORTED, "spectral transforms: nx, ny <= %d for this storage type (%d, %d)",
                    nmax, nx, ny);
    return IBM_OK;
}

size_t spectral_lds_bytes(const ibm_ctx* c, int n, int seqs, int threads) {
    const size_t cs = c->dtype == IBM_F64 ? 16 : 8;
    return ((size_t)team_lds_elems(threads) * seqs + (size_t)n) * cs;
}

long spectral_slots(const ibm_ctx* c) {
    // one per column group of a plane and drag component; none for a grid
    // the transforms refuse (its y pass would have no teams per block)
    if (!spectral_fits(c)) return 0;
    const int ny = c->g.ny, nx = c->g.nx;
    const int ty = (c->dtype == IBM_F64 ? kDyThreads<double> : kDyThreads<float>) / (ny >= 8 ? ny / 8 : 1);
    return 3L * ((nx + 2 * ty - 1) / (2 * ty)) * c->g.nz;
}

void free_spectral(ibm_ctx* c) { free_spectral_tables(c); }

int launch_apply_spectral(ibm_ctx* c, const void* const tau[6], void* const ustar[3],
                          const void* const gradp[3], double dt, void* const div[3],
                          double* drag, hipStream_t s) {
    if (c->dtype == IBM_F64) return spectral_t<double>(c, tau, ustar, gradp, dt, div, drag, s);
    return spectral_t<float>(c, tau, ustar, gradp, dt, div, drag, s);
}

}  // namespace ibm
