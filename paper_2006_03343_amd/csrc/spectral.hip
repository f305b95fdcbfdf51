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
//   k_dy   the same along y, a team per pair of columns of one plane, on
//          tau_xy + i tau_yy and tau_yz, adding d/dy tau_xy, d/dy tau_yy,
//          d/dy tau_yz and the staggered vertical differences (d/dz tau_xz,
//          tau_yz on uv nodes, d/dz tau_zz on w nodes, zero padded), loaded
//          with the divergence it updates; with the final divergence in hand
//          it leaves per-block drag partials over the fluid nodes, summed in
//          slot order by k_spec_finalize.
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

// Drag over the fluid nodes: flag bit 0 marks a forced uv node (div_x,
// div_y left out), bit 1 a forced w node (div_z left out).
template <typename Acc, typename T>
__device__ inline void drag_add(Acc (&acc)[3], uint32_t fb, T d0, T d1, T d2) {
    if (!(fb & 1u)) {
        acc[0] += (Acc)d0;
        acc[1] += (Acc)d1;
    }
    if (!(fb & 2u)) acc[2] += (Acc)d2;
}

// A team per pair of columns (c, c+1) of plane k; the teams of a block are
// interleaved across lanes (lane = j * teams + team), so a row's columns are
// read together.  A block's row segment (16 float columns, 64 B) is half a
// cache line whose other half the next block reads, and the vertical
// differences read the neighbouring planes' blocks' stresses: with the
// XCD-aware block order blocks that share lines run on one XCD's L2.  Sequences: tau_xy + i tau_yy of column c, of column c+1,
// and tau_yz of column c + i tau_yz of column c+1.  PAIR (float, nx even,
// fields 8-byte aligned): each field's two columns move as one 8-byte access.
template <typename T, bool ALL, bool PAIR, typename Acc>
__global__ void __launch_bounds__(256) k_dy(SpecArgs<T> a, ApplyArgs<T> z) {
    constexpr int G = kSeqAtOnce<T>;
    static_assert(!PAIR || G == 3, "column pairs move together only with all sequences at once");
    extern __shared__ unsigned char lds_raw[];
    Cx<T>* xl = reinterpret_cast<Cx<T>*>(lds_raw);
    const int n = a.ny, logn = a.logy;
    const int P = n >= 8 ? n >> 3 : 1, ns = n >= 8 ? 8 : n;
    const int teams = (int)blockDim.x / P;
    const int groups = (a.nx + 2 * teams - 1) / (2 * teams);
    const int lb = xcd_block(groups * a.nz);
    if (lb < 0) return;                                   // the whole block
    Cx<T>* tw = xl + team_lds_elems(blockDim.x) * (ALL ? G : 1);
    stage_twiddles(tw, a.twy, n);
    const int k = lb / groups;
    const int gi = lb - k * groups;
    const int team = (int)threadIdx.x % teams;
    const Team tm = make_team(logn, (int)threadIdx.x / teams, team, teams, true);
    const int c0 = 2 * (gi * teams + team);
    const bool in[2] = {c0 < a.nx, c0 + 1 < a.nx};
    const long pk = (long)k * a.ny * a.nx;
    Acc acc[3] = {Acc(0), Acc(0), Acc(0)};     // drag partials over the fluid nodes
    for (int s0 = 0; s0 < 3; s0 += G) {
        Cx<T> v[G][8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const long q = pk + (long)tm.elem(u) * a.nx + c0;
#pragma unroll
            for (int g = 0; g < G; ++g) v[g][u] = Cx<T>{T(0), T(0)};
            if (u >= ns) continue;
            if constexpr (PAIR) {
                if (!in[0]) continue;
                const Two<T> xy = *reinterpret_cast<const Two<T>*>(a.tau[3] + q);
                const Two<T> yy = *reinterpret_cast<const Two<T>*>(a.tau[1] + q);
                const Two<T> yz = *reinterpret_cast<const Two<T>*>(a.tau[5] + q);
                v[0][u] = Cx<T>{xy.x, yy.x};
                v[1][u] = Cx<T>{xy.y, yy.y};
                v[2][u] = Cx<T>{yz.x, yz.y};
            } else {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const int sq = s0 + g;
                    if (sq < 2) {
                        if (in[sq]) v[g][u] = Cx<T>{a.tau[3][q + sq], a.tau[1][q + sq]};
                    } else {
                        if (in[0]) v[g][u].re = a.tau[5][q];
                        if (in[1]) v[g][u].im = a.tau[5][q + 1];
                    }
                }
            }
        }
        __syncthreads();
        team_fft<T, G, ALL>(v, tm, xl, tw);
        derivative<T, G>(v, tm, n, a.ky);
        team_ifft<T, G, ALL>(v, tm, xl, tw);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (u >= ns) continue;
            const int row = tm.elem(u);
            const long q = pk + (long)row * a.nx + c0;
            // forcing flags of columns c0, c0 + 1 (one word: c0 is even)
            const uint32_t fw = (in[0] && s0 + G >= 3) ?
                z.fmask[((long)k * a.ny + row) * z.wrow + (c0 >> 4)] >> (2 * (c0 & 15)) : 0u;
            if constexpr (PAIR) {
                if (!in[0]) continue;
                Two<T>* d0 = reinterpret_cast<Two<T>*>(a.div[0] + q);
                Two<T>* d1 = reinterpret_cast<Two<T>*>(a.div[1] + q);
                Two<T>* d2 = reinterpret_cast<Two<T>*>(a.div[2] + q);
                const Two<T> o0 = *d0, o1 = *d1, o2 = *d2;
                // staggered vertical differences, loaded with the divergence
                const Two<T> zx = zdiff2(a, 4, q, k, true), zy = zdiff2(a, 5, q, k, true),
                             zz = zdiff2(a, 2, q, k, false);
                const Two<T> n0{o0.x + v[0][u].re + zx.x, o0.y + v[1][u].re + zx.y};
                const Two<T> n1{o1.x + v[0][u].im + zy.x, o1.y + v[1][u].im + zy.y};
                const Two<T> n2{o2.x + v[2][u].re + zz.x, o2.y + v[2][u].im + zz.y};
                *d0 = n0;
                *d1 = n1;
                *d2 = n2;
                drag_add(acc, fw, n0.x, n1.x, n2.x);
                if (in[1]) drag_add(acc, fw >> 2, n0.y, n1.y, n2.y);
            } else {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const int sq = s0 + g;
                    if (sq < 2) {
                        if (in[sq]) {
                            a.div[0][q + sq] += v[g][u].re;
                            a.div[1][q + sq] += v[g][u].im;
                        }
                    } else {
                        if (in[0]) a.div[2][q] += v[g][u].re;
                        if (in[1]) a.div[2][q + 1] += v[g][u].im;
                    }
                }
                if (s0 + G >= 3) {
                    // the last group: add the vertical differences, then
                    // every component of both columns is final
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        if (!in[h]) continue;
                        const long qh = q + h;
                        const T d0 = a.div[0][qh] + zdiff(a, 4, qh, k, true);
                        const T d1 = a.div[1][qh] + zdiff(a, 5, qh, k, true);
                        const T d2 = a.div[2][qh] + zdiff(a, 2, qh, k, false);
                        a.div[0][qh] = d0;
                        a.div[1][qh] = d1;
                        a.div[2][qh] = d2;
                        drag_add(acc, fw >> (2 * h), d0, d1, d2);
                    }
                }
            }
        }
    }
    if (!z.drag) return;
    __shared__ double red[3][4];
    const double w0 = wave_sum((double)acc[0]), w1 = wave_sum((double)acc[1]),
                 w2 = wave_sum((double)acc[2]);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wv] = w0;
        red[1][wv] = w1;
        red[2][wv] = w2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double r = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += red[threadIdx.x][w];
        z.partials[3L * lb + threadIdx.x] = r;
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
    const int ty = 256 / (ny >= 8 ? ny / 8 : 1);
    const int groups = (nx + 2 * ty - 1) / (2 * ty);
    const long nyb = (long)groups * nz;                     // y-pass blocks = drag slots
    if (c->ap_cap < 3L * nyb) return fail(IBM_E_STATE, "apply_spectral: reduction slots not sized");
    z.partials = c->ap_partials;
    z.nfblocks = (int)std::min<long>((4 * c->nfsegs + 7) / 8 * 8, 2048);
    const int tx = 256 / (nx >= 8 ? nx / 8 : 1);            // teams per block
    const long pairs = (a.rows + 1) / 2;
    const unsigned nrb = (unsigned)((pairs + tx - 1) / tx);
    // one sequence's exchange space: exchanging all three at once measured
    // slower here (more registers, fewer waves)
    hipLaunchKernelGGL((k_dx<T, false>), dim3(nrb + (unsigned)z.nfblocks), dim3(256),
                       spectral_lds_bytes(c, nx, 1), s, a, z, nrb);
    bool aligned = sizeof(T) == 4 && nx % 2 == 0;
    for (int i = 0; i < 6; ++i) aligned = aligned && (uintptr_t)tau[i] % (2 * sizeof(T)) == 0;
    for (int i = 0; i < 3; ++i) aligned = aligned && (uintptr_t)div[i] % (2 * sizeof(T)) == 0;
    const bool wide = c->precision == IBM_PREC_MIXED || sizeof(T) == 8;   // drag in double
    const dim3 gdy((unsigned)(8 * ((nyb + 7) / 8)));     // logical blocks dealt per XCD
    const size_t lds_y = spectral_lds_bytes(c, ny, 1);
    if (aligned && wide)
        hipLaunchKernelGGL((k_dy<T, false, sizeof(T) == 4, double>), gdy, dim3(256), lds_y, s, a, z);
    else if (aligned)
        hipLaunchKernelGGL((k_dy<T, false, sizeof(T) == 4, T>), gdy, dim3(256), lds_y, s, a, z);
    else if (wide)
        hipLaunchKernelGGL((k_dy<T, false, false, double>), gdy, dim3(256), lds_y, s, a, z);
    else
        hipLaunchKernelGGL((k_dy<T, false, false, T>), gdy, dim3(256), lds_y, s, a, z);
    if (drag)
        hipLaunchKernelGGL(k_spec_finalize, dim3(1), dim3(256), 0, s, (const double*)z.partials,
                           nyb, z.dv, drag);
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

size_t spectral_lds_bytes(const ibm_ctx* c, int n, int seqs) {
    const size_t cs = c->dtype == IBM_F64 ? 16 : 8;
    return ((size_t)team_lds_elems(256) * seqs + (size_t)n) * cs;
}

long spectral_slots(const ibm_ctx* c) {
    // one per y-pass block and drag component; none for a grid the
    // transforms refuse (its y pass would have no teams per block)
    if (!spectral_fits(c)) return 0;
    const int ny = c->g.ny, nx = c->g.nx;
    const int ty = 256 / (ny >= 8 ? ny / 8 : 1);
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
