// fft.h -- in-LDS radix-2 complex FFTs shared by the pseudo-spectral
// divergence (spectral.hip) and the pressure projection (projection.hip).
//
// A block transforms ``ns`` sequences of length n = 2^logn held in LDS, one
// after another.  The forward transform is decimation in time on
// bit-reversed input (natural-order output); the same forward transform by
// decimation in frequency takes natural-order input and leaves bit-reversed
// output, which gives an inverse as conj(FFT(conj X)) / n with no
// permutation pass.  Twiddles exp(-2 pi i t / n), t < n/2, come from a table
// the block stages into LDS.  Index arithmetic is shifts and masks.
#pragma once

#include <hip/hip_runtime.h>

namespace ibm {

template <typename T>
struct Cx {
    T re, im;
};

template <typename T>
__device__ inline Cx<T> cmul(Cx<T> a, Cx<T> b) {
    return Cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

__device__ inline unsigned bitrev(unsigned i, int logn) {
    return logn ? (__brev(i) >> (32 - logn)) : 0u;
}

// The twiddle table (n/2 entries) copied into LDS once per block.
template <typename T>
__device__ inline void stage_twiddles(Cx<T>* tl, const Cx<T>* __restrict__ tw, int n) {
    for (int t = threadIdx.x; t < n / 2; t += blockDim.x) tl[t] = tw[t];
}

// Forward FFT (decimation in time) of ``ns`` sequences of length n = 2^logn
// held in LDS in bit-reversed order, sequence s at s * n; natural-order
// output in place.  All threads of the block take part; index arithmetic is
// shifts and masks (n is a power of two); twiddles from the LDS table.
template <typename T>
__device__ void fft_dit(Cx<T>* x, int ns, int logn, const Cx<T>* tw) {
    if (logn == 0) return;
    const int lh = logn - 1, hmask = (1 << lh) - 1;
    const int nb = ns << lh;
    for (int s = 1; s <= logn; ++s) {
        const int ls = s - 1, half = 1 << ls;
        const int tsh = logn - s;            // W_{2 half}^pos = W_n^(pos << (logn - s))
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
            const int seq = b >> lh, bb = b & hmask;
            const int grp = bb >> ls, pos = bb & (half - 1);
            Cx<T>* base = x + (seq << logn) + (grp << s) + pos;
            const Cx<T> w = tw[pos << tsh];
            const Cx<T> a = base[0], t = cmul(w, base[half]);
            base[0] = Cx<T>{a.re + t.re, a.im + t.im};
            base[half] = Cx<T>{a.re - t.re, a.im - t.im};
        }
        __syncthreads();
    }
}

// Forward FFT (decimation in frequency) of natural-order input; the output
// lands in bit-reversed order.
template <typename T>
__device__ void fft_dif(Cx<T>* x, int ns, int logn, const Cx<T>* tw) {
    if (logn == 0) return;
    const int lh = logn - 1, hmask = (1 << lh) - 1;
    const int nb = ns << lh;
    for (int s = logn; s >= 1; --s) {
        const int ls = s - 1, half = 1 << ls;
        const int tsh = logn - s;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
            const int seq = b >> lh, bb = b & hmask;
            const int grp = bb >> ls, pos = bb & (half - 1);
            Cx<T>* base = x + (seq << logn) + (grp << s) + pos;
            const Cx<T> w = tw[pos << tsh];
            const Cx<T> a = base[0], c = base[half];
            base[0] = Cx<T>{a.re + c.re, a.im + c.im};
            base[half] = cmul(Cx<T>{a.re - c.re, a.im - c.im}, w);
        }
        __syncthreads();
    }
}

// X[m] -> conj(i k_m X[m] / n) for every sequence (natural order), k_m =
// 2 pi m' / L with m' = m or m - n, and 0 for the Nyquist mode.
template <typename T>
__device__ void derivative_conj(Cx<T>* x, int ns, int logn, T two_pi_over_len) {
    const int n = 1 << logn;
    const T inv_n = T(1) / T(n);
    for (int e = threadIdx.x; e < ns * n; e += blockDim.x) {
        const int m = e & (n - 1);
        const int mm = (2 * m < n) ? m : m - n;     // signed mode number (n = 1: mode 0)
        const T k = (n > 1 && 2 * m == n) ? T(0) : two_pi_over_len * T(mm) * inv_n;
        const Cx<T> v = x[e];
        // i k (re + i im) = -k im + i k re; then conjugate
        x[e] = Cx<T>{-k * v.im, -(k * v.re)};
    }
    __syncthreads();
}

}  // namespace ibm
