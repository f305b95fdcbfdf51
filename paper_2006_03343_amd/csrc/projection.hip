// projection.hip -- the AB2 update and the pressure projection that the
// paper's solver runs around the stage (§2.4, eqs. u-inter, u-t+1, p-Poisson,
// p-Poisson-Fourier).
//
// ibm_ab2_predict: u* = u + dt (3/2 RHS'^t - 1/2 RHS^(t - dt)), elementwise.
//
// ibm_pressure_project: by eq. dxdydz (dz = Lz / (nz - 1)) the w node 0 lies
// on the floor and the w node nz-1 on the lid; the uv layers 0 .. nz-2 are
// the cells between them and the uv layer nz-1 lies above the lid.  With D
// the discrete divergence of the spectral mode on the cells (pseudo-spectral
// d/dx, d/dy, (w[k+1] - w[k]) / dz) and G the discrete gradient
// (pseudo-spectral on uv nodes, (p[k] - p[k-1]) / dz on the interior w
// nodes), solve D G p = 2 / (3 dt) D u* with the wall w taken as 0 and set
// u = u* - (3 dt / 2) G p.  On the two wall w nodes the correction is the
// wall-normal gradient of eq. p-bc, 2 w* / (3 dt), which leaves w = 0 there
// (eqs. bc-bottom-u3, bc-top) and does not enter the cells' equations, so the
// wall nodes are written as 0.  In Fourier space along x and y each
// horizontal mode is one tridiagonal system over the nz - 1 cells:
//   p[k-1] / dz^2 - (K^2 + (number of neighbours) / dz^2) p[k] + p[k+1] / dz^2
//       = 2 / (3 dt) (i kx u_hat + i ky v_hat + (w_hat[k+1] - w_hat[k]) / dz),
// K^2 = kx^2 + ky^2 with Nyquist wavenumbers taken as 0; a mode with K = 0 is
// singular and takes p_hat = 0 at k = 0 in place of its first row (its
// right-hand sides sum to 0 with both walls at 0, so the system is
// consistent).  The layer above the lid gets p = 0 and keeps u*, v*.
//
// Real fields have Hermitian spectra along x, so only the modes 0 .. nx/2 are
// kept (rows padded to an even length).  Launches: k_rows_fwd -- forward x
// transforms of u*, v*, w*, two real rows packed into one complex transform
// and separated through the team's LDS; k_cols_fwd -- y transforms of pairs
// of half-spectrum columns, which leave the horizontal divergence spectrum
// H = i kx u_hat + i ky v_hat and w_hat; k_solve -- two threads per
// horizontal mode for the right-hand side 2 / (3 dt) (H + (w_hat[k+1] -
// w_hat[k]) / dz) and the tridiagonal system in z, eliminated from both ends
// (recurrences in double), leaving p_hat and its vertical difference
// p_hat[k] - p_hat[k-1]; k_cols_inv -- inverse y transforms of p_hat and
// i ky p_hat from one read, and of the vertical difference; k_rows_inv --
// inverse x transforms from the Hermitian extension, two rows per transform,
// returning p, u = u* - (3 dt / 2) d/dx p (i kx formed in the same pass),
// v = v* - (3 dt / 2) d/dy p and w = w* - (3 dt / 2) (p[k] - p[k-1]) / dz.
// Transforms: fft.h.
#include <algorithm>
#include <cmath>

#include "fft.h"
#include "kernels.h"

namespace ibm {
namespace {

template <typename T>
struct ProjArgs {
    int nx, ny, nz, logx, logy;
    int nh, nhp;             // x modes kept (nx/2 + 1) and the padded row length (even)
    long rows;               // ny * nz
    long plane;              // nx * ny
    long hplane;             // nhp * ny
    const Cx<T>* twx;
    const Cx<T>* twy;
    const T* in[3];          // u*, v*, w*
    Cx<T>* spec[3];          // their x spectra; then H and w_hat; p_hat and its vertical
                             // difference; P, DY and DZ
    const T* ub;             // u*, v*, w*: bases of the corrections
    const T* vb;
    const T* wb;
    T* uo;                   // u, v, w, p
    T* vo;
    T* wo;
    T* po;
    double kx, ky;           // 2 pi / Lx, 2 pi / Ly
    T kxs, kys;              // the same in the storage type
    double dz;
    double f;                // 2 / (3 dt)
    T c;                     // 3 dt / 2
    T dzs;                   // dz in the storage type, for the w correction
};

template <typename T>
__global__ void __launch_bounds__(256) k_ab2(const T* __restrict__ u, const T* __restrict__ rn,
                                             const T* __restrict__ rp, T dt, long n,
                                             T* __restrict__ out) {
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    out[q] = u[q] + dt * (T(1.5) * rn[q] - T(0.5) * rp[q]);
}

// Forward x transforms: a team of P = max(1, nx / 8) consecutive threads per
// pair of rows (r, r+1) of field blockIdx.y transforms Z = f_r + i f_{r+1};
// F_r = (Z_m + conj Z_{-m}) / 2 and F_{r+1} = (Z_m - conj Z_{-m}) / (2 i) for
// the modes m <= nx / 2.
template <typename T>
__global__ void __launch_bounds__(256) k_rows_fwd(ProjArgs<T> a) {
    extern __shared__ unsigned char lds_raw[];
    Cx<T>* xl = reinterpret_cast<Cx<T>*>(lds_raw);
    const int n = a.nx, logn = a.logx;
    const int P = n >= 8 ? n >> 3 : 1, ns = n >= 8 ? 8 : n;
    const int teams = (int)blockDim.x / P;
    Cx<T>* tw = xl + team_lds_elems(blockDim.x);
    stage_twiddles(tw, a.twx, n);
    const int team = (int)threadIdx.x / P;
    const Team tm = make_team(logn, (int)threadIdx.x - team * P, team, teams, false);
    const long r0 = 2 * ((long)blockIdx.x * teams + team);
    const bool in0 = r0 < a.rows, in1 = r0 + 1 < a.rows;
    const T* __restrict__ f = a.in[blockIdx.y];
    Cx<T>* __restrict__ out = a.spec[blockIdx.y];
    Cx<T> v[1][8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        v[0][u] = Cx<T>{T(0), T(0)};
        if (u >= ns) continue;
        const long o = r0 * n + tm.elem(u);
        v[0][u] = Cx<T>{in0 ? f[o] : T(0), in1 ? f[o + n] : T(0)};
    }
    __syncthreads();   // twiddles staged
    team_fft<T, 1>(v, tm, xl, tw);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u)
        if (u < ns) xl[tm.lds(tm.elem(u))] = v[0][u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int e = tm.elem(u);
        if (u >= ns || 2 * e > n) continue;
        const Cx<T> z = v[0][u], zc = xl[tm.lds((n - e) & (n - 1))];
        const T h = T(0.5);
        if (in0) out[r0 * a.nhp + e] = Cx<T>{h * (z.re + zc.re), h * (z.im - zc.im)};
        if (in1) out[(r0 + 1) * a.nhp + e] = Cx<T>{h * (z.im + zc.im), h * (zc.re - z.re)};
    }
}

// Inverse x transforms: a team per pair of rows builds Z_e = A_e + i B_e
// over all e from the half spectra A (row r) and B (row r+1) (A_e = conj
// A_{n-e} above nx / 2; the imaginary parts of modes 0 and nx / 2 are
// dropped, as a real inverse does) and inverts it.  blockIdx.y = 0: p from
// P; 1: u = u* - (3 dt / 2) d/dx p from i kx P; 2: v = v* - (3 dt / 2)
// d/dy p from DY; 3: w = w* - (3 dt / 2) (p[k] - p[k-1]) / dz from DZ, and
// w = 0 on the two wall planes.  One transform per team keeps the registers, and with them
// the waves per SIMD, of the forward x pass (two per team measured slower
// despite reading P once).
template <typename T, bool WT>
__global__ void __launch_bounds__(256) k_rows_inv(ProjArgs<T> a) {
    extern __shared__ unsigned char lds_raw[];
    Cx<T>* xl = reinterpret_cast<Cx<T>*>(lds_raw);
    const int n = a.nx, logn = a.logx;
    const int P = n >= 8 ? n >> 3 : 1, ns = WT ? 8 : n >= 8 ? 8 : n;
    const int teams = (int)blockDim.x / P;
    Cx<T>* tw = xl + team_lds_elems(blockDim.x);
    const int team = (int)threadIdx.x / P;
    const Team tm = make_team(logn, (int)threadIdx.x - team * P, team, teams, false);
    const int kind = (int)blockIdx.y;
    const long r0 = 2 * ((long)blockIdx.x * teams + team);
    const bool in0 = r0 < a.rows, in1 = r0 + 1 < a.rows;
    // rows past the end read the last row (in bounds, never stored): every load
    // is unconditional, so all of a thread's loads are in flight at once
    const long ca = in0 ? r0 : a.rows - 1, cb = in1 ? r0 + 1 : a.rows - 1;
    const Cx<T>* __restrict__ A = a.spec[kind < 2 ? 0 : kind - 1];
    // Slots above nx / 2 hold the conjugates of slots below it.  WT (a team's
    // threads lie in one wave, 8 <= nx <= 512): slots 5 .. 7 come from the
    // mirror thread P - j, slot 7 - u, through a lane permutation (thread 0
    // holds its own mirror, in slot 8 - u) instead of a second load of the
    // same lines.
    Cx<T> ra[8], rb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        ra[u] = rb[u] = Cx<T>{T(0), T(0)};
        if (u >= ns || (WT && u > 4)) continue;
        const int e = tm.elem(u);
        const int m = 2 * e > n ? n - e : e;
        ra[u] = A[ca * a.nhp + m];
        rb[u] = A[cb * a.nhp + m];
    }
    stage_twiddles(tw, a.twx, n);
    if constexpr (WT) {
        const int lane = (int)threadIdx.x & 63;
        const int src = lane - tm.j + ((P - tm.j) & (P - 1));
#pragma unroll
        for (int u = 5; u < 8; ++u) {
            const Cx<T> ma{__shfl(ra[7 - u].re, src), __shfl(ra[7 - u].im, src)};
            const Cx<T> mb{__shfl(rb[7 - u].re, src), __shfl(rb[7 - u].im, src)};
            ra[u] = tm.j == 0 ? ra[8 - u] : ma;
            rb[u] = tm.j == 0 ? rb[8 - u] : mb;
        }
    }
    Cx<T> v[1][8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        v[0][u] = Cx<T>{T(0), T(0)};
        if (u >= ns) continue;
        const int e = tm.elem(u);
        const bool upper = 2 * e > n;
        const int m = upper ? n - e : e;
        Cx<T> za = in0 ? ra[u] : Cx<T>{T(0), T(0)};
        Cx<T> zb = in1 ? rb[u] : Cx<T>{T(0), T(0)};
        if (m == 0 || 2 * m == n) {
            za.im = T(0);
            zb.im = T(0);
        }
        if (upper) {
            za.im = -za.im;
            zb.im = -zb.im;
        }
        if (kind == 1) {
            // i kx A + i (i kx B), kx signed, 0 at the Nyquist mode
            const T k = a.kxs * T(mode_number(e, n));
            v[0][u] = Cx<T>{-(k * za.im) - k * zb.re, k * za.re - k * zb.im};
        } else {
            v[0][u] = Cx<T>{za.re - zb.im, za.im + zb.re};
        }
    }
    __syncthreads();   // twiddles staged
    team_ifft<T, 1>(v, tm, xl, tw);
    T* out = kind == 0 ? a.po : kind == 1 ? a.uo : kind == 2 ? a.vo : a.wo;
    const T s = kind == 0 ? T(1) / T(n) : kind < 3 ? -a.c / T(n) : -a.c / (T(n) * a.dzs);
    // the bases of the corrections, all loads issued before the first store
    T b0[8], b1[8];
    if (kind) {
        const T* __restrict__ base = kind == 1 ? a.ub : kind == 2 ? a.vb : a.wb;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            b0[u] = b1[u] = T(0);
            if (u >= ns) continue;
            b0[u] = base[ca * n + tm.elem(u)];
            b1[u] = base[cb * n + tm.elem(u)];
        }
    }
    // rows are (k, j) pairs, k = r / ny: the w nodes on the floor and the lid are walls
    const long lid = (long)(a.nz - 1) * a.ny;
    const bool wall0 = kind == 3 && (r0 < a.ny || r0 >= lid);
    const bool wall1 = kind == 3 && (r0 + 1 < a.ny || r0 + 1 >= lid);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        if (u >= ns) continue;
        const long o = r0 * n + tm.elem(u);
        const T va = v[0][u].re * s, vb = v[0][u].im * s;
        if (in0) out[o] = wall0 ? T(0) : kind ? b0[u] + va : va;
        if (in1) out[o + n] = wall1 ? T(0) : kind ? b1[u] + vb : vb;
    }
}

// y transforms of the half spectra: a team per pair of adjacent columns of
// one plane, teams interleaved across lanes (lane = j * teams + team) so a
// row's columns are read together; a block's row segments straddle lines that
// the next block reads too, so the block order is XCD-aware.  Float moves both columns of a pair as
// one 16-byte access and transforms them together; double takes one column
// at a time (two would spill registers).
template <typename T>
struct alignas(2 * sizeof(Cx<T>)) CxPair {
    Cx<T> a, b;
};

template <typename T, int G>
__device__ inline void col_load(Cx<T> (&v)[G][8], const Cx<T>* base, const Team& tm, int nhp,
                                int ns, bool act) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
        for (int g = 0; g < G; ++g) v[g][u] = Cx<T>{T(0), T(0)};
        if (u >= ns || !act) continue;
        const Cx<T>* p = base + (long)tm.elem(u) * nhp;
        if constexpr (G == 2) {
            const CxPair<T> t = *reinterpret_cast<const CxPair<T>*>(p);
            v[0][u] = t.a;
            v[1][u] = t.b;
        } else {
            v[0][u] = *p;
        }
    }
}

template <typename T, int G>
__device__ inline void col_store(const Cx<T> (&v)[G][8], T scale, Cx<T>* base, const Team& tm,
                                 int nhp, int ns, bool act) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        if (u >= ns || !act) continue;
        Cx<T>* p = base + (long)tm.elem(u) * nhp;
        if constexpr (G == 2) {
            *reinterpret_cast<CxPair<T>*>(p) =
                CxPair<T>{Cx<T>{v[0][u].re * scale, v[0][u].im * scale},
                          Cx<T>{v[1][u].re * scale, v[1][u].im * scale}};
        } else {
            *p = Cx<T>{v[0][u].re * scale, v[0][u].im * scale};
        }
    }
}

// Signed x wavenumber of half-spectrum column i (0 at the Nyquist mode).
template <typename T>
__device__ inline T kx_of(const ProjArgs<T>& a, int i) {
    return (a.nx > 1 && 2 * i == a.nx) ? T(0) : a.kxs * T(i);
}

// Forward: u_hat, v_hat -> H = i kx u_hat + i ky v_hat (into spec[0]); w_hat
// in place.
template <typename T>
__global__ void __launch_bounds__(256) k_cols_fwd(ProjArgs<T> a) {
    constexpr int G = sizeof(T) == 4 ? 2 : 1;
    extern __shared__ unsigned char lds_raw[];
    Cx<T>* xl = reinterpret_cast<Cx<T>*>(lds_raw);
    const int n = a.ny, logn = a.logy;
    const int P = n >= 8 ? n >> 3 : 1, ns = n >= 8 ? 8 : n;
    const int teams = (int)blockDim.x / P;
    Cx<T>* tw = xl + team_lds_elems(blockDim.x) * G;
    stage_twiddles(tw, a.twy, n);
    const int cpairs = a.nhp / 2;
    const int groups = (cpairs + teams - 1) / teams;
    const int lb = xcd_block(groups * a.nz);
    if (lb < 0) return;                                   // the whole block
    const int k = lb / groups;
    const int gi = lb - k * groups;
    const int team = (int)threadIdx.x % teams;
    const Team tm = make_team(logn, (int)threadIdx.x / teams, team, teams, true);
    const int cp = gi * teams + team;
    const bool act = cp < cpairs;
    const long off = (long)k * a.hplane + 2 * cp;
    __syncthreads();   // twiddles staged
    for (int c = 0; c < 2; c += G) {
        Cx<T> hs[G][8], v[G][8];
        col_load<T, G>(v, a.spec[0] + off + c, tm, a.nhp, ns, act);
        team_fft<T, G, G == 2>(v, tm, xl, tw);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const T kx = kx_of(a, 2 * cp + c + g);
#pragma unroll
            for (int u = 0; u < 8; ++u) hs[g][u] = Cx<T>{-(kx * v[g][u].im), kx * v[g][u].re};
        }
        col_load<T, G>(v, a.spec[1] + off + c, tm, a.nhp, ns, act);
        team_fft<T, G, G == 2>(v, tm, xl, tw);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const T ky = a.kys * T(mode_number(tm.elem(u) & (n - 1), n));
#pragma unroll
            for (int g = 0; g < G; ++g) {
                hs[g][u].re -= ky * v[g][u].im;
                hs[g][u].im += ky * v[g][u].re;
            }
        }
        col_store<T, G>(hs, T(1), a.spec[0] + off + c, tm, a.nhp, ns, act);
        col_load<T, G>(v, a.spec[2] + off + c, tm, a.nhp, ns, act);
        team_fft<T, G, G == 2>(v, tm, xl, tw);
        col_store<T, G>(v, T(1), a.spec[2] + off + c, tm, a.nhp, ns, act);
    }
}

// Inverse: p_hat (spec[0]) -> P = its inverse y transform (in place) and
// DY = that of i ky p_hat (into spec[1]); then the vertical difference of
// p_hat (spec[2]) -> DZ, its inverse y transform (in place); all with 1 / ny.
template <typename T>
__global__ void __launch_bounds__(256) k_cols_inv(ProjArgs<T> a) {
    constexpr int G = sizeof(T) == 4 ? 2 : 1;
    extern __shared__ unsigned char lds_raw[];
    Cx<T>* xl = reinterpret_cast<Cx<T>*>(lds_raw);
    const int n = a.ny, logn = a.logy;
    const int P = n >= 8 ? n >> 3 : 1, ns = n >= 8 ? 8 : n;
    const int teams = (int)blockDim.x / P;
    Cx<T>* tw = xl + team_lds_elems(blockDim.x);
    stage_twiddles(tw, a.twy, n);
    const int cpairs = a.nhp / 2;
    const int groups = (cpairs + teams - 1) / teams;
    const int lb = xcd_block(groups * a.nz);
    if (lb < 0) return;                                   // the whole block
    const int k = lb / groups;
    const int gi = lb - k * groups;
    const int team = (int)threadIdx.x % teams;
    const Team tm = make_team(logn, (int)threadIdx.x / teams, team, teams, true);
    const int cp = gi * teams + team;
    const bool act = cp < cpairs;
    const long off = (long)k * a.hplane + 2 * cp;
    const T inv = T(1) / T(n);
    __syncthreads();   // twiddles staged
    for (int c = 0; c < 2; c += G) {
        Cx<T> pv[G][8];
        col_load<T, G>(pv, a.spec[0] + off + c, tm, a.nhp, ns, act);
        Cx<T> v[2 * G][8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const T ky = a.kys * T(mode_number(tm.elem(u) & (n - 1), n));
#pragma unroll
            for (int g = 0; g < G; ++g) {
                v[g][u] = pv[g][u];
                v[G + g][u] = Cx<T>{-(ky * pv[g][u].im), ky * pv[g][u].re};
            }
        }
        team_ifft<T, 2 * G>(v, tm, xl, tw);
        Cx<T> o[G][8];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int u = 0; u < 8; ++u) o[g][u] = v[g][u];
        col_store<T, G>(o, inv, a.spec[0] + off + c, tm, a.nhp, ns, act);
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int u = 0; u < 8; ++u) o[g][u] = v[G + g][u];
        col_store<T, G>(o, inv, a.spec[1] + off + c, tm, a.nhp, ns, act);
        col_load<T, G>(o, a.spec[2] + off + c, tm, a.nhp, ns, act);
        team_ifft<T, G>(o, tm, xl, tw);   // its first exchange waits for the block
        col_store<T, G>(o, inv, a.spec[2] + off + c, tm, a.nhp, ns, act);
    }
}

// Two threads per horizontal mode (i, j): the right-hand side and the
// tridiagonal system over the m = nz - 1 cells, eliminated from both ends at
// once, leaving p_hat in H's place.  Thread "top" runs Thomas forward
// elimination over rows 0 .. h-1 (h = m / 2), leaving p_k = d'_k - c'_k
// p_{k+1}; thread "bottom" eliminates rows m-1 .. h+1 upward, leaving p_k =
// d''_k - a''_k p_{k-1}, and forms row h's right-hand side.  Through LDS each
// gets the other's last coefficients and both solve row h with the same
// expression, then substitute back over their own rows.  A mode's chain is
// thus half as long and twice as many threads hide the memory latency.  The
// wall w values (levels 0 and nz-1) enter as 0; the level above the lid gets
// p_hat = 0.
//
// The recurrences run in double whatever the storage type: a K = 0 system is
// a Neumann chain pinned at one end whose condition number grows as nz^2, and
// float arithmetic in them over a few hundred levels loses the digits the
// transforms keep (rounding only the stored coefficients to float costs
// ~1e-7).  Each level's coefficient goes into the real part of H and its d
// into W, once that level's own values (and, going up, the w above it) have
// been read; row h is written by the top thread only after the exchange.
constexpr int kSolveModes = 128;    // modes per block; blockDim = 2 * kSolveModes

template <typename T>
__global__ void __launch_bounds__(256) k_solve(ProjArgs<T> a) {
    __shared__ double xs[8][kSolveModes];
    Cx<T>* __restrict__ H = a.spec[0];
    Cx<T>* __restrict__ W = a.spec[2];
    const int lane = (int)threadIdx.x % kSolveModes;
    const bool top = (int)threadIdx.x < kSolveModes;
    const long mode = (long)blockIdx.x * kSolveModes + lane;
    const int i = (int)(mode % a.nhp), j = (int)(mode / a.nhp);
    const bool act = mode < a.hplane && i < a.nh;
    auto wavenumber = [](int m, int n, double k0) {
        if (n > 1 && 2 * m == n) return 0.0;                // Nyquist
        return k0 * (double)(2 * m < n ? m : m - n);
    };
    const double kx = wavenumber(i, a.nx, a.kx), ky = wavenumber(j, a.ny, a.ky);
    const double K2 = kx * kx + ky * ky;
    const double e = 1.0 / (a.dz * a.dz);
    const double invdz = 1.0 / a.dz;
    const int m = a.nz - 1, h = m / 2;                       // cells; the meeting row
    const bool pin = K2 == 0.0;
    const long hp = a.hplane;
    const Cx<T> zero{T(0), T(0)};
    if (m < 1) {                                             // nz = 1: no cell
        if (act && !top) {
            H[mode] = zero;
            W[mode] = zero;
        }
        return;
    }
    // 2 / (3 dt) (H + (w[k+1] - w[k]) / dz)
    auto rhs = [&](Cx<T> hh, Cx<T> w, Cx<T> wu) {
        return Cx<double>{a.f * ((double)hh.re + ((double)wu.re - (double)w.re) * invdz),
                          a.f * ((double)hh.im + ((double)wu.im - (double)w.im) * invdz)};
    };
    if (top) {
        // rows 0 .. h-1, the next level's loads issued before this level's work;
        // the floor's w (level 0) is 0 and level h + 1 <= m - 1 is below the lid
        double cT = 0.0;
        Cx<double> dT{0.0, 0.0};
        if (act && h > 0) {
            Cx<T> hn = H[mode], wn = zero, wun = W[hp + mode];
            for (int k = 0; k < h; ++k) {
                const long q = (long)k * hp + mode;
                const Cx<T> hh = hn, w = wn, wu = wun;
                if (k + 1 < h) {
                    hn = H[q + hp];
                    wn = wu;
                    wun = W[q + 2 * hp];                    // k + 2 <= h < m
                }
                Cx<double> r = rhs(hh, w, wu);
                const double lo = k > 0 ? e : 0.0;
                double up = e, b = -K2 - lo - e;            // k + 1 <= h < m
                if (pin && k == 0) {
                    b = 1.0;
                    up = 0.0;
                    r = Cx<double>{0.0, 0.0};
                }
                const double rm = 1.0 / (b - lo * cT);
                cT = up * rm;
                dT = Cx<double>{(r.re - lo * dT.re) * rm, (r.im - lo * dT.im) * rm};
                W[q] = Cx<T>{(T)dT.re, (T)dT.im};
                H[q].re = (T)cT;
            }
        }
        xs[0][lane] = cT;
        xs[1][lane] = dT.re;
        xs[2][lane] = dT.im;
    } else {
        // rows m-1 .. h+1 going up (the lid's w above row m-1 is 0), then row
        // h's right-hand side
        double aB = 0.0;
        Cx<double> dB{0.0, 0.0}, rh{0.0, 0.0};
        if (act) {
            Cx<T> wu = zero;                                 // original w one level up
            const long qt = (long)(m - 1) * hp + mode;
            Cx<T> hn = H[qt], wn = m - 1 > 0 ? W[qt] : zero;
            for (int k = m - 1; k > h; --k) {
                const long q = (long)k * hp + mode;
                const Cx<T> hh = hn, w = wn;
                hn = H[q - hp];                              // k - 1 >= h
                wn = k - 1 > 0 ? W[q - hp] : zero;           // the floor's w is 0
                const Cx<double> r = rhs(hh, w, wu);
                const double up = k + 1 < m ? e : 0.0;
                const double b = -K2 - e - up;               // k >= 1
                const double rm = 1.0 / (b - up * aB);
                aB = e * rm;
                dB = Cx<double>{(r.re - up * dB.re) * rm, (r.im - up * dB.im) * rm};
                W[q] = Cx<T>{(T)dB.re, (T)dB.im};
                H[q].re = (T)aB;
                wu = w;
            }
            rh = rhs(hn, wn, wu);                            // row h, from the originals
        }
        xs[3][lane] = aB;
        xs[4][lane] = dB.re;
        xs[5][lane] = dB.im;
        xs[6][lane] = rh.re;
        xs[7][lane] = rh.im;
    }
    __syncthreads();
    if (!act) return;
    // row h: lo p_{h-1} + b p_h + up p_{h+1} = r_h with p_{h-1} = d'_{h-1} -
    // c'_{h-1} p_h and p_{h+1} = d''_{h+1} - a''_{h+1} p_h
    const double cT = xs[0][lane], aB = xs[3][lane];
    const Cx<double> dT{xs[1][lane], xs[2][lane]}, dB{xs[4][lane], xs[5][lane]};
    Cx<double> r{xs[6][lane], xs[7][lane]};
    const double lo = h > 0 ? e : 0.0;
    double up = h + 1 < m ? e : 0.0, b = -K2 - lo - up;
    if (pin && h == 0) {
        b = 1.0;
        up = 0.0;
        r = Cx<double>{0.0, 0.0};
    }
    const double rm = 1.0 / (b - lo * cT - up * aB);
    const Cx<double> ph{(r.re - lo * dT.re - up * dB.re) * rm, (r.im - lo * dT.im - up * dB.im) * rm};
    auto coef = [&](long q, Cx<double>& d, double& c) {
        const Cx<T> t = W[q];
        d = Cx<double>{(double)t.re, (double)t.im};
        c = (double)H[q].re;
    };
    // Back substitution.  Besides p_hat (into H) each level leaves the
    // vertical difference p_hat[k] - p_hat[k-1] of the w correction, formed
    // here in double (into W, whose d' it has read): the small-K modes carry a
    // large part nearly constant in z that a difference of stored float
    // pressures would cancel badly.  W on the wall levels 0 and nz-1 is 0 (the
    // inverse x pass writes w = 0 there), as are p_hat and W above the lid.
    auto diff = [&](long q, const Cx<double>& hi, const Cx<double>& lo_) {
        W[q] = Cx<T>{(T)(hi.re - lo_.re), (T)(hi.im - lo_.im)};
    };
    Cx<double> p = ph, dn;
    double cn;
    if (top) {
        H[(long)h * hp + mode] = Cx<T>{(T)ph.re, (T)ph.im};
        if (h > 0) coef((long)(h - 1) * hp + mode, dn, cn);
        for (int k = h - 1; k >= 0; --k) {
            const long q = (long)k * hp + mode;
            const Cx<double> d = dn;
            const double c = cn;
            if (k > 0) coef(q - hp, dn, cn);
            const Cx<double> pk{d.re - c * p.re, d.im - c * p.im};
            H[q] = Cx<T>{(T)pk.re, (T)pk.im};
            diff(q + hp, p, pk);                             // level k + 1 <= h
            p = pk;
        }
        W[mode] = zero;                                      // level 0
    } else {
        if (h + 1 < m) coef((long)(h + 1) * hp + mode, dn, cn);
        for (int k = h + 1; k < m; ++k) {
            const long q = (long)k * hp + mode;
            const Cx<double> d = dn;
            const double c = cn;
            if (k + 1 < m) coef(q + hp, dn, cn);
            const Cx<double> pk{d.re - c * p.re, d.im - c * p.im};
            H[q] = Cx<T>{(T)pk.re, (T)pk.im};
            diff(q, pk, p);                                  // level k > h
            p = pk;
        }
        const long ql = (long)m * hp + mode;                 // level nz-1: lid / above it
        H[ql] = zero;
        W[ql] = zero;
    }
}

inline unsigned nb256(long n) { return (unsigned)((n + 255) / 256); }

template <typename T>
int project_t(ibm_ctx* c, const void* const ustar[3], double dt, void* const uo[3], void* p_out,
              hipStream_t s) {
    int rc = spectral_check(c);
    if (rc) return rc;
    if ((rc = ensure_twiddles(c))) return rc;
    ProjArgs<T> a;
    a.nx = c->g.nx;
    a.ny = c->g.ny;
    a.nz = c->g.nz;
    a.logx = 0;
    while ((1 << a.logx) < a.nx) ++a.logx;
    a.logy = 0;
    while ((1 << a.logy) < a.ny) ++a.logy;
    a.nh = a.nx / 2 + 1;
    a.nhp = (a.nh + 1) & ~1;
    a.rows = (long)a.ny * a.nz;
    a.plane = (long)a.nx * a.ny;
    a.hplane = (long)a.nhp * a.ny;
    const long nspec = a.hplane * a.nz;
    if (!c->proj.buf) {
        const size_t cb = sizeof(Cx<T>) * (size_t)nspec;
        IBM_HIP(hipMalloc(&c->proj.buf, 3 * cb));
        c->proj.bytes = 3 * cb;
    }
    Cx<T>* U = (Cx<T>*)c->proj.buf;
    Cx<T>* V = U + nspec;
    Cx<T>* W = V + nspec;
    a.twx = (const Cx<T>*)c->spec.twx;
    a.twy = (const Cx<T>*)c->spec.twy;
    a.kx = 2.0 * M_PI / (a.nx * c->g.dx);
    a.ky = 2.0 * M_PI / (a.ny * c->g.dy);
    a.dz = c->g.dz;
    a.f = 2.0 / (3.0 * dt);
    a.c = (T)(1.5 * dt);
    a.dzs = (T)c->g.dz;
    Cx<T>* spec[3] = {U, V, W};
    for (int i = 0; i < 3; ++i) {
        a.in[i] = (const T*)ustar[i];
        a.spec[i] = spec[i];
    }
    a.ub = (const T*)ustar[0];
    a.vb = (const T*)ustar[1];
    a.wb = (const T*)ustar[2];
    a.uo = (T*)uo[0];
    a.vo = (T*)uo[1];
    a.wo = (T*)uo[2];
    a.po = (T*)p_out;
    a.kxs = (T)a.kx;
    a.kys = (T)a.ky;
    const int tx = 256 / (a.nx >= 8 ? a.nx / 8 : 1);     // teams per block
    const int ty = 256 / (a.ny >= 8 ? a.ny / 8 : 1);
    const unsigned gx = (unsigned)(((a.rows + 1) / 2 + tx - 1) / tx);
    const long ncb = (long)((a.nhp / 2 + ty - 1) / ty) * a.nz;   // column blocks
    const unsigned gy = (unsigned)(8 * ((ncb + 7) / 8));          // dealt per XCD
    constexpr int G = sizeof(T) == 4 ? 2 : 1;            // columns per y-transform phase
    hipLaunchKernelGGL(k_rows_fwd<T>, dim3(gx, 3), dim3(256), spectral_lds_bytes(c, a.nx, 1), s, a);
    hipLaunchKernelGGL(k_cols_fwd<T>, dim3(gy), dim3(256), spectral_lds_bytes(c, a.ny, G), s, a);
    hipLaunchKernelGGL(k_solve<T>, dim3((unsigned)((a.hplane + kSolveModes - 1) / kSolveModes)),
                       dim3(2 * kSolveModes), 0, s, a);
    hipLaunchKernelGGL(k_cols_inv<T>, dim3(gy), dim3(256), spectral_lds_bytes(c, a.ny, 1), s, a);
    // p, u = u* - c d/dx p, v = v* - c d/dy p, w = w* - c (p[k] - p[k-1]) / dz
    if (a.nx >= 8 && a.nx <= 512)
        hipLaunchKernelGGL((k_rows_inv<T, true>), dim3(gx, 4), dim3(256),
                           spectral_lds_bytes(c, a.nx, 1), s, a);
    else
        hipLaunchKernelGGL((k_rows_inv<T, false>), dim3(gx, 4), dim3(256),
                           spectral_lds_bytes(c, a.nx, 1), s, a);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

template <typename T>
int ab2_t(ibm_ctx* c, const void* const u[3], const void* const rn[3], const void* const rp[3],
          double dt, void* const out[3], hipStream_t s) {
    for (int i = 0; i < 3; ++i)
        hipLaunchKernelGGL(k_ab2<T>, dim3(nb256(c->n)), dim3(256), 0, s, (const T*)u[i],
                           (const T*)rn[i], (const T*)rp[i], (T)dt, c->n, (T*)out[i]);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

}  // namespace

int launch_pressure_project(ibm_ctx* c, const void* const ustar[3], double dt,
                            void* const u_out[3], void* p_out, hipStream_t s) {
    if (c->dtype == IBM_F64) return project_t<double>(c, ustar, dt, u_out, p_out, s);
    return project_t<float>(c, ustar, dt, u_out, p_out, s);
}

int launch_ab2(ibm_ctx* c, const void* const u[3], const void* const rhs_now[3],
               const void* const rhs_prev[3], double dt, void* const ustar[3], hipStream_t s) {
    if (c->dtype == IBM_F64) return ab2_t<double>(c, u, rhs_now, rhs_prev, dt, ustar, s);
    return ab2_t<float>(c, u, rhs_now, rhs_prev, dt, ustar, s);
}

void free_projection(ibm_ctx* c) {
    (void)hipFree(c->proj.buf);
    c->proj.buf = nullptr;
    c->proj.bytes = 0;
}

}  // namespace ibm
