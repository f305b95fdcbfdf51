// fft.h -- register-resident complex FFTs for thread teams, shared by the
// pseudo-spectral divergence (spectral.hip) and the pressure projection
// (projection.hip).
//
// Stockham autosort formulation (Govindaraju et al., SC 2008): a sequence of
// n = 2^logn complex values is transformed by a team of P = max(1, n / 8)
// threads.  Thread j of the team holds element j + u P of the sequence in
// register slot u (u < 8; u < n when n < 8), in natural order before and
// after the transform, so a transform starts from coalesced loads, ends in
// coalesced stores, and a forward transform followed by a pointwise product
// and another transform needs no exchange in between.
//
// Passes: one of radix 2 or 4 first when logn is not a multiple of 3, then
// radix 8.  A pass of radix r over span Ns (the product of the radices before
// it) is run by n / r virtual threads v, each taking inputs v + m n / r
// (m < r), multiplying input m by W_n^(m k n / (Ns r)) with k = v mod Ns, an
// r-point DFT, and writing output m to (v - k) r + k + m Ns.  Thread j runs
// the virtual threads j + t P (t < 8 / r), whose inputs and -- in the last
// pass -- outputs are exactly its own slots; between passes the team exchanges
// through LDS.
//
// LDS: element e of a team's sequence lives at (e + e / 2^ps) * se + off;
// rows (teams of consecutive lanes) take se = 1, ps = 4, off = team * (n +
// n / 16), columns (teams interleaved across lanes) se = teams per block,
// ps = 3, off = team.  The padding breaks the strides of the exchanges'
// writes (first pass: 8 consecutive elements per thread); one in 16 for rows
// (one in 8 before) cut the spectral x pass's LDS bank conflicts (0.523
// against 0.540 ms per spectral call, identical results), while columns keep
// one in 8 (0.5 % faster projection than one in 16).
// Twiddles W_n^t, t < n, come from a table (computed in double on the host)
// the block stages into LDS.
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
template <typename T>
__device__ inline Cx<T> cadd(Cx<T> a, Cx<T> b) {
    return Cx<T>{a.re + b.re, a.im + b.im};
}
template <typename T>
__device__ inline Cx<T> csub(Cx<T> a, Cx<T> b) {
    return Cx<T>{a.re - b.re, a.im - b.im};
}
template <typename T>
__device__ inline Cx<T> mul_mi(Cx<T> a) {   // -i a
    return Cx<T>{a.im, -a.re};
}

// A team's place in the block and its LDS addressing.
struct Team {
    int j;       // thread's index in the team, 0 .. P - 1
    int logn;    // n = 2^logn
    int P;       // threads per team
    int se;      // LDS stride between consecutive (padded) elements
    int off;     // LDS offset of the team's element 0
    int ps;      // padding: one empty element after every 2^ps
    __device__ int lds(int e) const { return (e + (e >> ps)) * se + off; }
    __device__ int elem(int u) const { return j + u * P; }   // element held in slot u
};

// LDS elements a block of ``threads`` threads needs for its teams' exchanges.
inline __host__ __device__ int team_lds_elems(int threads) { return threads * 9; }

__device__ inline Team make_team(int logn, int j, int team, int teams, bool columns) {
    const int n = 1 << logn;
    Team t;
    t.j = j;
    t.logn = logn;
    t.P = n >= 8 ? n >> 3 : 1;
    t.se = columns ? teams : 1;
    t.ps = columns ? 3 : 4;
    t.off = columns ? team : team * (n + (n >> 4));
    return t;
}

template <typename T>
__device__ inline void stage_twiddles(Cx<T>* tl, const Cx<T>* __restrict__ tw, int n) {
    for (int t = threadIdx.x; t < n; t += blockDim.x) tl[t] = tw[t];
}

template <typename T>
__device__ inline void dft2(Cx<T>& a0, Cx<T>& a1) {
    const Cx<T> t = a0;
    a0 = cadd(t, a1);
    a1 = csub(t, a1);
}

template <typename T>
__device__ inline void dft4(Cx<T>& a0, Cx<T>& a1, Cx<T>& a2, Cx<T>& a3) {
    const Cx<T> t0 = cadd(a0, a2), t1 = csub(a0, a2);
    const Cx<T> t2 = cadd(a1, a3), t3 = mul_mi(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

// 8-point DFT, natural order in and out: two 4-point DFTs of the even and odd
// inputs joined with W_8^k.
template <typename T>
__device__ inline void dft8(Cx<T> (&a)[8]) {
    dft4(a[0], a[2], a[4], a[6]);
    dft4(a[1], a[3], a[5], a[7]);
    const T h = T(0.70710678118654752440084436210484904);   // sqrt(1/2)
    const Cx<T> o1{h * (a[3].re + a[3].im), h * (a[3].im - a[3].re)};     // W_8^1 O_1
    const Cx<T> o2 = mul_mi(a[5]);                                        // W_8^2 O_2
    const Cx<T> o3{h * (a[7].im - a[7].re), -h * (a[7].re + a[7].im)};    // W_8^3 O_3
    const Cx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6], o0 = a[1];
    a[0] = cadd(e0, o0);
    a[4] = csub(e0, o0);
    a[1] = cadd(e1, o1);
    a[5] = csub(e1, o1);
    a[2] = cadd(e2, o2);
    a[6] = csub(e2, o2);
    a[3] = cadd(e3, o3);
    a[7] = csub(e3, o3);
}

template <typename T, int RAD>
__device__ inline void dft_r(Cx<T> (&a)[RAD]) {
    if constexpr (RAD == 2) dft2(a[0], a[1]);
    else if constexpr (RAD == 4) dft4(a[0], a[1], a[2], a[3]);
    else dft8(a);
}

// One pass in registers: the virtual threads j + t P (t < 8 / RAD) of span Ns.
template <typename T, int RAD, int S>
__device__ inline void pass_regs(Cx<T> (&v)[S][8], const Team& tm, int Ns, int log_step,
                                 const Cx<T>* tw) {
    constexpr int VT = 8 / RAD;
#pragma unroll
    for (int t = 0; t < VT; ++t) {
        const int k = (tm.j + t * tm.P) & (Ns - 1);
        Cx<T> w[RAD];
#pragma unroll
        for (int m = 1; m < RAD; ++m) w[m] = tw[(m * k) << log_step];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            Cx<T> a[RAD];
#pragma unroll
            for (int m = 0; m < RAD; ++m) a[m] = v[s][t + m * VT];
            if (Ns > 1) {
#pragma unroll
                for (int m = 1; m < RAD; ++m) a[m] = cmul(a[m], w[m]);
            }
            dft_r<T, RAD>(a);
#pragma unroll
            for (int m = 0; m < RAD; ++m) v[s][t + m * VT] = a[m];
        }
    }
}

// The outputs of a pass of radix RAD and span Ns (not the last pass) go to
// LDS and come back as the next pass's slots: all S sequences at once when
// ALL (sequence s at s * team_lds_elems(blockDim.x)), else one at a time
// through one sequence's space.
template <typename T, int RAD, int S, bool ALL>
__device__ inline void pass_exchange(Cx<T> (&v)[S][8], const Team& tm, int Ns, Cx<T>* lds) {
    constexpr int VT = 8 / RAD;
    constexpr int NB = ALL ? 1 : S;             // rounds
    constexpr int PR = ALL ? S : 1;             // sequences per round
    const int sst = team_lds_elems(blockDim.x);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        __syncthreads();
#pragma unroll
        for (int t = 0; t < VT; ++t) {
            const int vv = tm.j + t * tm.P;
            const int k = vv & (Ns - 1);
            const int e0 = (vv - k) * RAD + k;
#pragma unroll
            for (int m = 0; m < RAD; ++m) {
                const int a = tm.lds(e0 + m * Ns);
#pragma unroll
                for (int r = 0; r < PR; ++r) lds[a + r * sst] = v[b * PR + r][t + m * VT];
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int a = tm.lds(tm.elem(u));
#pragma unroll
            for (int r = 0; r < PR; ++r) v[b * PR + r][u] = lds[a + r * sst];
        }
    }
}

// Forward DFT (exponent -2 pi i) of S sequences held in the team's slots.
// Every thread of the block must call it (it synchronises the block) with the
// same logn.  LDS: team_lds_elems(blockDim.x) elements, times S when ALL.
template <typename T, int S, bool ALL = false>
__device__ void team_fft(Cx<T> (&v)[S][8], const Team& tm, Cx<T>* lds, const Cx<T>* tw) {
    const int logn = tm.logn;
    if (logn < 3) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (logn == 1) dft2(v[s][0], v[s][1]);
            else if (logn == 2) dft4(v[s][0], v[s][1], v[s][2], v[s][3]);
        }
        return;
    }
    const int r0 = logn % 3;
    int Ns = 1, lspan = 0;                      // lspan = log2(Ns)
    if (r0 == 1) {
        pass_regs<T, 2, S>(v, tm, Ns, logn - 1, tw);
        pass_exchange<T, 2, S, ALL>(v, tm, Ns, lds);
        Ns = 2;
        lspan = 1;
    } else if (r0 == 2) {
        pass_regs<T, 4, S>(v, tm, Ns, logn - 2, tw);
        pass_exchange<T, 4, S, ALL>(v, tm, Ns, lds);
        Ns = 4;
        lspan = 2;
    }
    for (int p = 0; p < logn / 3; ++p) {
        pass_regs<T, 8, S>(v, tm, Ns, logn - lspan - 3, tw);
        if (lspan + 3 < logn) pass_exchange<T, 8, S, ALL>(v, tm, Ns, lds);
        Ns <<= 3;
        lspan += 3;
    }
}

// The inverse DFT without the 1/n factor, through the forward one:
// sum X_m exp(+2 pi i m e / n) = swap(FFT(swap(X))) with swap(a + ib) = b + ia.
template <typename T, int S>
__device__ inline void swap_parts(Cx<T> (&v)[S][8]) {
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int u = 0; u < 8; ++u) v[s][u] = Cx<T>{v[s][u].im, v[s][u].re};
}

template <typename T, int S, bool ALL = false>
__device__ void team_ifft(Cx<T> (&v)[S][8], const Team& tm, Cx<T>* lds, const Cx<T>* tw) {
    swap_parts(v);
    team_fft<T, S, ALL>(v, tm, lds, tw);
    swap_parts(v);
}

// Signed mode number of element m of a sequence of n: m or m - n; the
// Nyquist mode of an even n is reported as 0 (it takes no derivative).
__device__ inline int mode_number(int m, int n) {
    if (n > 1 && 2 * m == n) return 0;
    return 2 * m < n ? m : m - n;
}

}  // namespace ibm
