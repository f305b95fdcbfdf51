// projection.hip -- the AB2 update and the pressure projection that the
// paper's solver runs around the stage (§2.4, eqs. u-inter, u-t+1, p-Poisson,
// p-Poisson-Fourier).
//
// ibm_ab2_predict: u* = u + dt (3/2 RHS'^t - 1/2 RHS^(t - dt)), elementwise.
//
// ibm_pressure_project: with D the discrete divergence of the spectral mode
// (pseudo-spectral d/dx, d/dy on uv nodes, (w[k+1] - w[k]) / dz with w above
// the top node taken as 0) and G the discrete gradient (pseudo-spectral on uv
// nodes, (p[k] - p[k-1]) / dz on w nodes k >= 1, none on the bottom w node),
// solve D G p = 2 / (3 dt) D u* and set u = u* - (3 dt / 2) G p.  In Fourier
// space along x and y each horizontal mode is one tridiagonal system in z:
//   p[k-1] / dz^2 - (K^2 + (number of neighbours) / dz^2) p[k] + p[k+1] / dz^2
//       = 2 / (3 dt) (i kx u_hat + i ky v_hat + (w_hat[k+1] - w_hat[k]) / dz),
// K^2 = kx^2 + ky^2 with Nyquist wavenumbers taken as 0; a mode with K = 0 is
// singular and takes p_hat = 0 at k = 0 in place of its first row.  The
// projected field is then discretely divergence-free wherever the singular
// modes are solvable (e.g. w = 0 on the bottom plane).
//
// Launches: forward x transforms of u*, v*, w* (real rows -> complex), forward
// y transforms (complex columns, in place), one thread per horizontal mode
// for the right-hand side, a Thomas sweep in z (in double) and the gradient spectra
// i kx p_hat, i ky p_hat, p_hat (coalesced across modes), inverse y
// transforms, inverse x transforms that apply the horizontal corrections to
// u and v and return p, and the vertical correction of w.  Transforms: fft.h.
#include <algorithm>
#include <cmath>

#include "fft.h"
#include "kernels.h"

namespace ibm {
namespace {

template <typename T>
struct ProjArgs {
    int nx, ny, nz, logx, logy;
    long rows;               // ny * nz
    long plane;
    int rows_per, cols;      // per transform block
    const Cx<T>* twx;
    const Cx<T>* twy;
    double kx, ky;           // 2 pi / Lx, 2 pi / Ly
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

// Forward x transform of R real rows per block into complex rows (natural
// order).
template <typename T>
__global__ void __launch_bounds__(256) k_rows_fwd(ProjArgs<T> a, const T* __restrict__ f,
                                                  Cx<T>* __restrict__ out) {
    extern __shared__ unsigned char lds_raw[];
    Cx<T>* x = reinterpret_cast<Cx<T>*>(lds_raw);
    const int n = a.nx, logn = a.logx, R = a.rows_per;
    Cx<T>* tw = x + R * n;
    stage_twiddles(tw, a.twx, n);
    const long r0 = (long)R * blockIdx.x;
    for (int e = threadIdx.x; e < R * n; e += blockDim.x) {
        const int r = e >> logn, i = e & (n - 1);
        const bool in = r0 + r < a.rows;
        x[(r << logn) + bitrev((unsigned)i, logn)] =
            Cx<T>{in ? f[(r0 + r) * n + i] : T(0), T(0)};
    }
    __syncthreads();
    fft_dit(x, R, logn, tw);
    for (int e = threadIdx.x; e < R * n; e += blockDim.x) {
        const int r = e >> logn, i = e & (n - 1);
        if (r0 + r < a.rows) out[(r0 + r) * n + i] = x[e];
    }
}

// Inverse x transform of R complex rows per block (natural order); the real
// result, times ``scale``, is added to ``base`` (or stored if base is null).
template <typename T>
__global__ void __launch_bounds__(256) k_rows_inv(ProjArgs<T> a, const Cx<T>* __restrict__ in,
                                                  const T* base, T scale, T* out) {
    extern __shared__ unsigned char lds_raw[];
    Cx<T>* x = reinterpret_cast<Cx<T>*>(lds_raw);
    const int n = a.nx, logn = a.logx, R = a.rows_per;
    Cx<T>* tw = x + R * n;
    stage_twiddles(tw, a.twx, n);
    const long r0 = (long)R * blockIdx.x;
    for (int e = threadIdx.x; e < R * n; e += blockDim.x) {
        const int r = e >> logn;
        const Cx<T> v = r0 + r < a.rows ? in[r0 * n + e] : Cx<T>{T(0), T(0)};
        x[e] = Cx<T>{v.re, -v.im};                         // conj
    }
    __syncthreads();
    fft_dif(x, R, logn, tw);
    const T s = scale / T(n);
    for (int e = threadIdx.x; e < R * n; e += blockDim.x) {
        const int r = e >> logn, i = e & (n - 1);
        if (r0 + r >= a.rows) continue;
        const long o = (r0 + r) * n + i;
        // inverse = conj(FFT(conj X)) / n; its real part is the bit-reversed
        // output's real part
        const T v = x[(r << logn) + bitrev((unsigned)i, logn)].re * s;
        out[o] = base ? base[o] + v : v;
    }
}

// y transform in place of C complex columns of one plane per block; inverse
// includes the 1/ny factor.
template <typename T>
__global__ void __launch_bounds__(256) k_cols(ProjArgs<T> a, Cx<T>* __restrict__ data,
                                              int inverse) {
    extern __shared__ unsigned char lds_raw[];
    Cx<T>* x = reinterpret_cast<Cx<T>*>(lds_raw);
    const int n = a.ny, logn = a.logy, C = a.cols;
    Cx<T>* tw = x + C * n;
    stage_twiddles(tw, a.twy, n);
    const int groups = (a.nx + C - 1) / C;
    const int k = blockIdx.x / groups;
    const int x0 = (blockIdx.x - k * groups) * C;
    const long pk = (long)k * a.plane;
    for (int e = threadIdx.x; e < C * n; e += blockDim.x) {
        const int c = e % C, j = e / C;
        const bool in = x0 + c < a.nx;
        const Cx<T> v = in ? data[pk + (long)j * a.nx + x0 + c] : Cx<T>{T(0), T(0)};
        if (inverse) x[c * n + j] = Cx<T>{v.re, -v.im};
        else x[c * n + bitrev((unsigned)j, logn)] = v;
    }
    __syncthreads();
    if (inverse) fft_dif(x, C, logn, tw);
    else fft_dit(x, C, logn, tw);
    const T s = T(1) / T(n);
    for (int e = threadIdx.x; e < C * n; e += blockDim.x) {
        const int c = e % C, j = e / C;
        if (x0 + c >= a.nx) continue;
        Cx<T>& d = data[pk + (long)j * a.nx + x0 + c];
        if (inverse) {
            const Cx<T> v = x[c * n + bitrev((unsigned)j, logn)];
            d = Cx<T>{v.re * s, -v.im * s};
        } else {
            d = x[c * n + j];
        }
    }
}

// One thread per horizontal mode (i, j): right-hand side, Thomas sweep in z,
// then U = i kx p_hat, V = i ky p_hat, W = p_hat.  The sweep runs in double whatever the
// storage type.  A K = 0 system is a Neumann chain pinned at one end whose
// condition number grows as nz^2, so a float sweep over a few hundred levels
// would lose the digits the transforms keep.  The forward sweep stores d' and
// c' in the slots of the level it has just read: with float storage each
// complex slot of U, V, W is 8 bytes, one double (d'.re in U, d'.im in V, c'
// in W); with double storage d' goes into W and c' into cp.
template <typename T>
__global__ void __launch_bounds__(256) k_solve(ProjArgs<T> a, Cx<T>* __restrict__ U,
                                               Cx<T>* __restrict__ V, Cx<T>* __restrict__ W,
                                               double* __restrict__ cp) {
    constexpr bool narrow = sizeof(T) == 4;
    const long mode = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (mode >= a.plane) return;
    const int i = (int)(mode % a.nx), j = (int)(mode / a.nx);
    auto wavenumber = [](int m, int n, double k0) {
        if (n > 1 && 2 * m == n) return 0.0;                // Nyquist
        return k0 * (double)(2 * m < n ? m : m - n);
    };
    const double kx = wavenumber(i, a.nx, a.kx), ky = wavenumber(j, a.ny, a.ky);
    const double K2 = kx * kx + ky * ky;
    const double e = 1.0 / (a.dz * a.dz);
    const double invdz = 1.0 / a.dz;
    const int nz = a.nz;
    const bool pin = K2 == 0.0;
    double* const dre = (double*)U;
    double* const dim = (double*)V;
    double* const cw = (double*)W;
    // forward sweep; level k's slots are rewritten once W[k] and W[k+1] have been read
    Cx<double> dprev{0.0, 0.0};
    double cprev = 0.0;
    for (int k = 0; k < nz; ++k) {
        const long q = (long)k * a.plane + mode;
        const Cx<T> u = U[q], v = V[q], w = W[q];
        const Cx<T> wu = k + 1 < nz ? W[q + a.plane] : Cx<T>{T(0), T(0)};
        // i kx u + i ky v + (w[k+1] - w[k]) / dz
        Cx<double> r{-(kx * (double)u.im) - ky * (double)v.im + ((double)wu.re - (double)w.re) * invdz,
                     kx * (double)u.re + ky * (double)v.re + ((double)wu.im - (double)w.im) * invdz};
        r.re *= a.f;
        r.im *= a.f;
        double lo = k > 0 ? e : 0.0, up = k + 1 < nz ? e : 0.0;
        double b = -K2 - lo - up;
        if (pin && k == 0) {
            b = 1.0;
            up = 0.0;
            r = Cx<double>{0.0, 0.0};
        }
        const double m = b - lo * cprev;
        const double cn = up / m;
        const Cx<double> dn{(r.re - lo * dprev.re) / m, (r.im - lo * dprev.im) / m};
        if constexpr (narrow) {
            dre[q] = dn.re;
            dim[q] = dn.im;
            cw[q] = cn;
        } else {
            W[q] = Cx<T>{dn.re, dn.im};
            cp[q] = cn;
        }
        cprev = cn;
        dprev = dn;
    }
    // back substitution and the gradient spectra
    Cx<double> pnext{0.0, 0.0};
    for (int k = nz - 1; k >= 0; --k) {
        const long q = (long)k * a.plane + mode;
        Cx<double> d;
        double cc;
        if constexpr (narrow) {
            d = Cx<double>{dre[q], dim[q]};
            cc = cw[q];
        } else {
            const Cx<T> t = W[q];
            d = Cx<double>{(double)t.re, (double)t.im};
            cc = cp[q];
        }
        const Cx<double> p{d.re - cc * pnext.re, d.im - cc * pnext.im};
        W[q] = Cx<T>{(T)p.re, (T)p.im};
        U[q] = Cx<T>{(T)(-(kx * p.im)), (T)(kx * p.re)};
        V[q] = Cx<T>{(T)(-(ky * p.im)), (T)(ky * p.re)};
        pnext = p;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_wcorr(ProjArgs<T> a, const T* __restrict__ ws,
                                               const T* __restrict__ p, T* __restrict__ wo) {
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.plane * a.nz) return;
    const T v = ws[q];
    wo[q] = q >= a.plane ? v - a.c * ((p[q] - p[q - a.plane]) / a.dzs) : v;
}

inline unsigned nb256(long n) { return (unsigned)((n + 255) / 256); }

template <typename T>
int project_t(ibm_ctx* c, const void* const ustar[3], double dt, void* const uo[3], void* p_out,
              hipStream_t s) {
    int R = 2, C = 2;
    int rc = spectral_plan(c, &R, &C);
    if (rc) return rc;
    if ((rc = ensure_twiddles(c))) return rc;
    const long n = c->n;
    if (!c->proj.buf) {
        // float storage keeps the sweep's doubles in the three spectra
        const size_t cb = sizeof(Cx<T>) * (size_t)n;
        const size_t rb = sizeof(T) == 8 ? sizeof(double) * (size_t)n : 0;
        IBM_HIP(hipMalloc(&c->proj.buf, 3 * cb + rb));
        c->proj.bytes = 3 * cb + rb;
    }
    Cx<T>* U = (Cx<T>*)c->proj.buf;
    Cx<T>* V = U + n;
    Cx<T>* W = V + n;
    double* cp = sizeof(T) == 8 ? (double*)(W + n) : nullptr;
    ProjArgs<T> a;
    a.nx = c->g.nx;
    a.ny = c->g.ny;
    a.nz = c->g.nz;
    a.logx = 0;
    while ((1 << a.logx) < a.nx) ++a.logx;
    a.logy = 0;
    while ((1 << a.logy) < a.ny) ++a.logy;
    a.rows = (long)a.ny * a.nz;
    a.plane = (long)a.nx * a.ny;
    a.rows_per = R;
    a.cols = C;
    a.twx = (const Cx<T>*)c->spec.twx;
    a.twy = (const Cx<T>*)c->spec.twy;
    a.kx = 2.0 * M_PI / (a.nx * c->g.dx);
    a.ky = 2.0 * M_PI / (a.ny * c->g.dy);
    a.dz = c->g.dz;
    a.f = 2.0 / (3.0 * dt);
    a.c = (T)(1.5 * dt);
    a.dzs = (T)c->g.dz;
    const size_t lx = ((size_t)R * a.nx + a.nx / 2) * sizeof(Cx<T>);
    const size_t ly = ((size_t)C * a.ny + a.ny / 2) * sizeof(Cx<T>);
    const unsigned gx = (unsigned)((a.rows + R - 1) / R);
    const unsigned gy = (unsigned)(((a.nx + C - 1) / C) * a.nz);
    Cx<T>* spec[3] = {U, V, W};
    for (int i = 0; i < 3; ++i) {
        hipLaunchKernelGGL(k_rows_fwd<T>, dim3(gx), dim3(256), lx, s, a, (const T*)ustar[i], spec[i]);
        hipLaunchKernelGGL(k_cols<T>, dim3(gy), dim3(256), ly, s, a, spec[i], 0);
    }
    hipLaunchKernelGGL(k_solve<T>, dim3(nb256(a.plane)), dim3(256), 0, s, a, U, V, W, cp);
    for (int i = 0; i < 3; ++i)
        hipLaunchKernelGGL(k_cols<T>, dim3(gy), dim3(256), ly, s, a, spec[i], 1);
    // u = u* - c d/dx p, v = v* - c d/dy p, then p itself
    hipLaunchKernelGGL(k_rows_inv<T>, dim3(gx), dim3(256), lx, s, a, (const Cx<T>*)U,
                       (const T*)ustar[0], -a.c, (T*)uo[0]);
    hipLaunchKernelGGL(k_rows_inv<T>, dim3(gx), dim3(256), lx, s, a, (const Cx<T>*)V,
                       (const T*)ustar[1], -a.c, (T*)uo[1]);
    hipLaunchKernelGGL(k_rows_inv<T>, dim3(gx), dim3(256), lx, s, a, (const Cx<T>*)W,
                       (const T*)nullptr, T(1), (T*)p_out);
    hipLaunchKernelGGL(k_wcorr<T>, dim3(nb256(n)), dim3(256), 0, s, a, (const T*)ustar[2],
                       (const T*)p_out, (T*)uo[2]);
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
