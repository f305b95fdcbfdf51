// spectral.hip -- the stress divergence with the paper's own pseudo-spectral
// horizontal derivatives (§2.4, eq. dudx) instead of central differences:
//   d/dx A = sum over wavenumbers of i k A_hat exp(i k x), periodic in x and
//   y, the Nyquist mode of an even node count without derivative; the
//   vertical staggered differences (eqs. dudz, dwdz), the forcing (eq.
//   u-*-IBM) and the drag are those of the dense pass.
//
// Three launches, each HBM bound:
//   k_dx   one block per R rows (up to 8, as LDS allows): complex FFTs of
//          length nx in LDS on tau_xx + i tau_xy of each row and tau_xz of
//          two rows packed into one sequence (the derivative is a real operator, so the real and
//          imaginary parts stay separate); multiply by i k / nx with the
//          Nyquist mode dropped (explicitly: with two fields packed its term
//          would leak into the other field); inverse transform; write
//          div_x = d/dx tau_xx, div_y = d/dx tau_xy, div_z = d/dx tau_xz;
//   k_dy   one block per C consecutive columns of one plane: the same along
//          y on tau_xy + i tau_yy and on tau_yz of two columns, adding
//          d/dy tau_xy, d/dy tau_yy, d/dy tau_yz;
//   k_spec_z  adds the staggered vertical differences, leaves per-block drag
//          partials (finalized in slot order), and forces the forcing
//          segments in the blocks after the dense ones.
// Transform: iterative radix-2; the forward one is decimation in time on
// bit-reversed input (natural-order output), the inverse one decimation in
// frequency on natural-order input computed as conj(FFT(conj X)), so its
// output is read back at bit-reversed positions and no permutation pass is
// needed.  Twiddles exp(-2 pi i t / N), t < N/2, come from a table computed
// in double on the host and staged into LDS by each block.
#include <algorithm>
#include <cmath>
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
    int cols;                // columns per k_dy block (even)
    int rows_per;            // rows per k_dx block (even)
    T kx, ky;                // 2 pi / Lx, 2 pi / Ly
};

// R rows per block (R even): sequence r = tau_xx + i tau_xy of row r0 + r,
// sequence R + r/2 = tau_xz of rows r0 + r (real part, r even) and r0 + r + 1
// (imaginary part); the twiddle table follows the sequences in LDS.
template <typename T>
__global__ void __launch_bounds__(256) k_dx(SpecArgs<T> a) {
    extern __shared__ unsigned char lds_raw[];
    Cx<T>* x = reinterpret_cast<Cx<T>*>(lds_raw);
    const int n = a.nx, logn = a.logx, R = a.rows_per;
    const int ns = R + R / 2;
    Cx<T>* tw = x + ns * n;
    stage_twiddles(tw, a.twx, n);
    const long r0 = (long)R * blockIdx.x;
    for (int e = threadIdx.x; e < R * n; e += blockDim.x) {
        const int r = e >> logn, i = e & (n - 1);
        const bool in = r0 + r < a.rows;
        const long o = (r0 + r) * n + i;
        const unsigned p = bitrev((unsigned)i, logn);
        x[(r << logn) + p] = in ? Cx<T>{a.tau[0][o], a.tau[3][o]} : Cx<T>{T(0), T(0)};
        const T xz = in ? a.tau[4][o] : T(0);
        Cx<T>& q = x[((R + r / 2) << logn) + p];
        if (r & 1) q.im = xz;
        else q.re = xz;
    }
    __syncthreads();
    fft_dit(x, ns, logn, tw);
    derivative_conj(x, ns, logn, a.kx);
    fft_dif(x, ns, logn, tw);
    // the derivative at i is conj(x[bitrev(i)]): real part x.re, imaginary -x.im
    for (int e = threadIdx.x; e < R * n; e += blockDim.x) {
        const int r = e >> logn, i = e & (n - 1);
        if (r0 + r >= a.rows) continue;
        const long o = (r0 + r) * n + i;
        const unsigned p = bitrev((unsigned)i, logn);
        const Cx<T> d = x[(r << logn) + p];
        const Cx<T> dq = x[((R + r / 2) << logn) + p];
        a.div[0][o] = d.re;
        a.div[1][o] = -d.im;
        a.div[2][o] = (r & 1) ? -dq.im : dq.re;
    }
}

// C columns (x0 .. x0+C-1) of plane k per block: sequences c = tau_xy + i
// tau_yy of column c, and C + c/2 = tau_yz of columns c, c+1 (C even).
template <typename T>
__global__ void __launch_bounds__(256) k_dy(SpecArgs<T> a) {
    extern __shared__ unsigned char lds_raw[];
    Cx<T>* x = reinterpret_cast<Cx<T>*>(lds_raw);
    const int n = a.ny, logn = a.logy, C = a.cols;
    Cx<T>* tw = x + (C + C / 2) * n;
    stage_twiddles(tw, a.twy, n);
    const int groups = (a.nx + C - 1) / C;
    const int k = blockIdx.x / groups;
    const int x0 = (blockIdx.x - k * groups) * C;
    const long pk = (long)k * a.ny * a.nx;
    // thread t: column t % C, rows t / C, t / C + 256 / C, ...  (coalesced in x)
    for (int e = threadIdx.x; e < C * n; e += blockDim.x) {
        const int c = e % C, j = e / C;
        const int xx = x0 + c;
        const bool in = xx < a.nx;
        const long q = pk + (long)j * a.nx + (in ? xx : 0);
        const unsigned p = bitrev((unsigned)j, logn);
        x[c * n + p] = in ? Cx<T>{a.tau[3][q], a.tau[1][q]} : Cx<T>{T(0), T(0)};
        const T yz = in ? a.tau[5][q] : T(0);
        Cx<T>& s = x[(C + c / 2) * n + p];
        if (c & 1) s.im = yz;
        else s.re = yz;
    }
    __syncthreads();
    const int ns = C + C / 2;
    fft_dit(x, ns, logn, tw);
    derivative_conj(x, ns, logn, a.ky);
    fft_dif(x, ns, logn, tw);
    for (int e = threadIdx.x; e < C * n; e += blockDim.x) {
        const int c = e % C, j = e / C;
        const int xx = x0 + c;
        if (xx >= a.nx) continue;
        const long q = pk + (long)j * a.nx + xx;
        const unsigned p = bitrev((unsigned)j, logn);
        const Cx<T> d = x[c * n + p];
        const Cx<T> dz = x[(C + c / 2) * n + p];
        a.div[0][q] += d.re;
        a.div[1][q] += -d.im;
        a.div[2][q] += (c & 1) ? -dz.im : dz.re;
    }
}

// Vertical staggered differences added to the horizontal parts, drag
// partials per block (3 slots), then forcing in the blocks after the dense
// ones (quarters of the forcing segments).
constexpr int kZItems = 8;

template <typename T, typename Acc>
__global__ void __launch_bounds__(256) k_spec_z(ApplyArgs<T> a, int nzb) {
    if ((int)blockIdx.x >= nzb) {
        constexpr int kPiece = kSeg / 4;
        for (long it = blockIdx.x - nzb; it < 4 * a.nfsegs; it += a.nfblocks) {
            const Seg sg = a.fsegs[it >> 2];
            const int off = (int)(it & 3) * kPiece;
            if (off < sg.len)
                force_seg<T>(a, Seg{sg.q + off, min(kPiece, sg.len - off), 0, 0}, threadIdx.x,
                             blockDim.x);
        }
        return;
    }
    __shared__ double red[3][4];
    // 32-bit offsets: a context holds fewer than 2^31 nodes
    const int plane = (int)a.plane;
    const int n = plane * a.nz;
    Acc s0 = Acc(0), s1 = Acc(0), s2 = Acc(0);
    const int q0 = blockIdx.x * blockDim.x * kZItems + threadIdx.x;
    for (int it = 0; it < kZItems; ++it) {
        const int q = q0 + it * blockDim.x;
        if (q >= n) break;
        const int k = q / plane;
        const int rem = q - k * plane;
        const int row = rem / a.nx;
        const int xi = rem - row * a.nx;
        const T xz_up = k + 1 < a.nz ? a.tau[4][q + plane] : T(0);
        const T yz_up = k + 1 < a.nz ? a.tau[5][q + plane] : T(0);
        const T zz_dn = k > 0 ? a.tau[2][q - plane] : T(0);
        const T d0 = a.div[0][q] + (xz_up - a.tau[4][q]) * a.cz;
        const T d1 = a.div[1][q] + (yz_up - a.tau[5][q]) * a.cz;
        const T d2 = a.div[2][q] + (a.tau[2][q] - zz_dn) * a.cz;
        a.div[0][q] = d0;
        a.div[1][q] = d1;
        a.div[2][q] = d2;
        const uint32_t fb = a.fmask[(k * a.ny + row) * a.wrow + (xi >> 4)] >> (2 * (xi & 15));
        if (!(fb & 1u)) {
            s0 += (Acc)d0;
            s1 += (Acc)d1;
        }
        if (!(fb & 2u)) s2 += (Acc)d2;
    }
    if (!a.drag) return;
    const double w0 = wave_sum((double)s0), w1 = wave_sum((double)s1), w2 = wave_sum((double)s2);
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
        a.partials[3L * blockIdx.x + threadIdx.x] = r;
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

size_t lds_limit() { return 64 * 1024; }   // dynamic LDS a block may take without an attribute

template <typename T>
int twiddles(ibm_ctx* c, int n, void** dst) {
    std::vector<Cx<T>> t(std::max(1, n / 2));
    for (int i = 0; i < n / 2; ++i) {
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
    const size_t cs = sizeof(Cx<T>);
    int R = 2, C = 2;
    int rc0 = spectral_plan(c, &R, &C);
    if (rc0) return rc0;
    int rc = ensure_twiddles(c);
    if (rc) return rc;
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
    a.cols = C;
    a.rows_per = R;
    a.kx = (T)(2.0 * M_PI / (nx * c->g.dx));
    a.ky = (T)(2.0 * M_PI / (ny * c->g.dy));
    hipLaunchKernelGGL(k_dx<T>, dim3((unsigned)((a.rows + R - 1) / R)), dim3(256),
                       ((size_t)(R + R / 2) * nx + nx / 2) * cs, s, a);
    const int groups = (nx + C - 1) / C;
    hipLaunchKernelGGL(k_dy<T>, dim3((unsigned)(groups * nz)), dim3(256),
                       ((size_t)(C + C / 2) * ny + ny / 2) * cs, s, a);
    ApplyArgs<T> z = make_apply_args<T>(c, c->cfg, tau, ustar, gradp, dt, div, drag);
    const long n = c->n;
    const int nzb = (int)((n + 256L * kZItems - 1) / (256L * kZItems));
    if (c->ap_cap < 3L * nzb) return fail(IBM_E_STATE, "apply_spectral: reduction slots not sized");
    z.partials = c->ap_partials;
    z.nfblocks = (int)std::min<long>((4 * c->nfsegs + 7) / 8 * 8, 2048);
    const unsigned grid = (unsigned)(nzb + z.nfblocks);
    if (c->precision == IBM_PREC_MIXED || sizeof(T) == 8)
        hipLaunchKernelGGL((k_spec_z<T, double>), dim3(grid), dim3(256), 0, s, z, nzb);
    else
        hipLaunchKernelGGL((k_spec_z<T, float>), dim3(grid), dim3(256), 0, s, z, nzb);
    if (drag)
        hipLaunchKernelGGL(k_spec_finalize, dim3(1), dim3(256), 0, s, (const double*)z.partials,
                           (long)nzb, z.dv, drag);
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

int spectral_plan(const ibm_ctx* c, int* rows_per, int* cols) {
    const int nx = c->g.nx, ny = c->g.ny;
    const size_t cs = c->dtype == IBM_F64 ? 16 : 8;
    if (ilog2_exact(nx) < 0 || ilog2_exact(ny) < 0)
        return fail(IBM_E_UNSUPPORTED, "spectral transforms: nx and ny must be powers of two (%d, %d)",
                    nx, ny);
    auto fits = [&](int seqs, int n) { return ((size_t)seqs * n + n / 2) * cs <= lds_limit(); };
    int R = 8;
    while (R > 2 && !fits(R + R / 2, nx)) R /= 2;
    if (!fits(R + R / 2, nx))
        return fail(IBM_E_UNSUPPORTED, "spectral transforms: nx = %d too long for one block's LDS", nx);
    int C = 64;
    while (C > 2 && !fits(C + C / 2, ny)) C /= 2;
    if (!fits(C + C / 2, ny))
        return fail(IBM_E_UNSUPPORTED, "spectral transforms: ny = %d too long for one block's LDS", ny);
    *rows_per = R;
    *cols = std::min(C, std::max(2, nx));
    return IBM_OK;
}

long spectral_slots(const ibm_ctx* c) {
    return 3 * ((c->n + 256L * kZItems - 1) / (256L * kZItems));
}

void free_spectral(ibm_ctx* c) { free_spectral_tables(c); }

int launch_apply_spectral(ibm_ctx* c, const void* const tau[6], void* const ustar[3],
                          const void* const gradp[3], double dt, void* const div[3],
                          double* drag, hipStream_t s) {
    if (c->dtype == IBM_F64) return spectral_t<double>(c, tau, ustar, gradp, dt, div, drag, s);
    return spectral_t<float>(c, tau, ustar, gradp, dt, div, drag, s);
}

}  // namespace ibm
