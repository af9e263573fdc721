// Self-sorting (Stockham) mixed-radix FFT building blocks for lines held in
// LDS.  One pass of radix R over a line of length N, with Ls the product of
// the radices already applied, maps butterfly j (k = j mod Ls):
//     v_r = x[j + r N/R] * w^(r k),  w = exp(s 2 pi i / (Ls R)),
//     v   = DFT_R(v),
//     y[(j - k) R + k + r Ls] = v_r,
// and after the last pass the line holds its DFT in natural order.  The
// sign s is -1 for the forward and +1 for the inverse transform.  Passes run
// in place: every thread reads all its inputs, the block synchronises, then
// every thread writes its outputs.
#pragma once

#include "common.hpp"

namespace sdf {

template <int... R>
struct Radices {};

// radix schedules; threads per line = N / 8 for every size
template <int N>
struct DefaultPlan;
template <>
struct DefaultPlan<8> { using type = Radices<8>; };
template <>
struct DefaultPlan<16> { using type = Radices<4, 4>; };
template <>
struct DefaultPlan<32> { using type = Radices<8, 4>; };
template <>
struct DefaultPlan<64> { using type = Radices<8, 8>; };
template <>
struct DefaultPlan<96> { using type = Radices<8, 4, 3>; };
template <>
struct DefaultPlan<128> { using type = Radices<8, 4, 4>; };

template <int N>
struct FFTShape {
    static constexpr int TPL = N / 8;  // threads per line
};

// ---------------------------------------------------------------- small DFTs
template <typename T, int S>
__device__ __forceinline__ void dft2(cplx<T>* v) {
    cplx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
}
template <typename T, int S>
__device__ __forceinline__ void dft3(cplx<T>* v) {
    const T h = T(0.86602540378443864676);  // sqrt(3) / 2
    cplx<T> t = v[1] + v[2];
    cplx<T> d = v[1] - v[2];
    cplx<T> u = mul_i<T, S>(d) * h;
    cplx<T> m = v[0] - t * T(0.5);
    v[0] = v[0] + t;
    v[1] = m + u;
    v[2] = m - u;
}
template <typename T, int S>
__device__ __forceinline__ void dft4(cplx<T>* v) {
    cplx<T> t0 = v[0] + v[2], t1 = v[0] - v[2];
    cplx<T> t2 = v[1] + v[3], t3 = mul_i<T, S>(v[1] - v[3]);
    v[0] = t0 + t2;
    v[2] = t0 - t2;
    v[1] = t1 + t3;
    v[3] = t1 - t3;
}
template <typename T, int S>
__device__ __forceinline__ void dft8(cplx<T>* v) {
    const T r = T(0.70710678118654752440);
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<T, S>(e);
    dft4<T, S>(o);
    // w8^1 = (1 + s i)/sqrt2, w8^2 = s i, w8^3 = (-1 + s i)/sqrt2
    cplx<T> o1 = (o[1] + mul_i<T, S>(o[1])) * r;
    cplx<T> o2 = mul_i<T, S>(o[2]);
    cplx<T> o3 = (mul_i<T, S>(o[3]) - o[3]) * r;
    v[0] = e[0] + o[0];
    v[4] = e[0] - o[0];
    v[1] = e[1] + o1;
    v[5] = e[1] - o1;
    v[2] = e[2] + o2;
    v[6] = e[2] - o2;
    v[3] = e[3] + o3;
    v[7] = e[3] - o3;
}
// v * (c + s S i): multiplication by a unit root given by its cosine and
// the magnitude of its sine
template <typename T, int S>
__device__ __forceinline__ cplx<T> rot_by(cplx<T> v, T c, T s) {
    const T ss = S > 0 ? s : -s;
    return mk(v.re * c - v.im * ss, v.re * ss + v.im * c);
}
// 16 = 4 x 4: DFT4 over n1 of x[4 n1 + n2], twiddle by w16^(n2 k1), DFT4
// over n2; output k1 + 4 k2
template <typename T, int S>
__device__ __forceinline__ void dft16(cplx<T>* v) {
    const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173), r = T(0.70710678118654752440);
    cplx<T> a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = v[4 * n1 + n2];
        dft4<T, S>(a[n2]);
    }
    a[1][1] = rot_by<T, S>(a[1][1], c1, s1);   // w^1
    a[1][2] = rot_by<T, S>(a[1][2], r, r);     // w^2
    a[1][3] = rot_by<T, S>(a[1][3], s1, c1);   // w^3
    a[2][1] = rot_by<T, S>(a[2][1], r, r);     // w^2
    a[2][2] = mul_i<T, S>(a[2][2]);            // w^4
    a[2][3] = rot_by<T, S>(a[2][3], -r, r);    // w^6
    a[3][1] = rot_by<T, S>(a[3][1], s1, c1);   // w^3
    a[3][2] = rot_by<T, S>(a[3][2], -r, r);    // w^6
    a[3][3] = rot_by<T, S>(a[3][3], -c1, -s1); // w^9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cplx<T> b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
        dft4<T, S>(b);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = b[k2];
    }
}
// 12 = 4 x 3: DFT4 over n1 of x[3 n1 + n2], twiddle by w12^(n2 k1), DFT3
// over n2; output k1 + 4 k2
template <typename T, int S>
__device__ __forceinline__ void dft12(cplx<T>* v) {
    const T h = T(0.86602540378443864676), q = T(0.5);  // cos 30 deg, sin 30 deg
    cplx<T> a[3][4];
#pragma unroll
    for (int n2 = 0; n2 < 3; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) a[n2][n1] = v[3 * n1 + n2];
        dft4<T, S>(a[n2]);
    }
    a[1][1] = rot_by<T, S>(a[1][1], h, q);   // w^1
    a[1][2] = rot_by<T, S>(a[1][2], q, h);   // w^2
    a[1][3] = mul_i<T, S>(a[1][3]);          // w^3
    a[2][1] = rot_by<T, S>(a[2][1], q, h);   // w^2
    a[2][2] = rot_by<T, S>(a[2][2], -q, h);  // w^4
    a[2][3] = mk(-a[2][3].re, -a[2][3].im);  // w^6
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cplx<T> b[3] = {a[0][k1], a[1][k1], a[2][k1]};
        dft3<T, S>(b);
#pragma unroll
        for (int k2 = 0; k2 < 3; ++k2) v[k1 + 4 * k2] = b[k2];
    }
}
template <typename T, int S, int R>
__device__ __forceinline__ void dftR(cplx<T>* v) {
    if constexpr (R == 2) dft2<T, S>(v);
    else if constexpr (R == 3) dft3<T, S>(v);
    else if constexpr (R == 4) dft4<T, S>(v);
    else if constexpr (R == 8) dft8<T, S>(v);
    else if constexpr (R == 12) dft12<T, S>(v);
    else if constexpr (R == 16) dft16<T, S>(v);
}

// Twiddle table tw[m] = exp(-2 pi i m / N), m < N, filled by the whole block.
template <typename T, int N>
__device__ __forceinline__ void fill_twiddles(cplx<T>* tw) {
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        double s, c;
        sincospi(-2.0 * double(m) / double(N), &s, &c);
        tw[m] = mk(T(c), T(s));
    }
}

// One Stockham pass over `CONC` lines at once.  Thread (line, t): line
// element e is at buf[line * ls + e * es].  Every thread of the block must
// call this (inactive threads pass active = false) because it synchronises.
template <typename T, int N, int S, int R, int LS, int TPL>
__device__ __forceinline__ void stockham_pass(cplx<T>* line_base, int es, int t, bool active,
                                              const cplx<T>* tw) {
    constexpr int NB = N / R;
    constexpr int PER = (NB + TPL - 1) / TPL;
    cplx<T> v[PER][R];
    if (active) {
#pragma unroll
        for (int b = 0; b < PER; ++b) {
            int j = t + b * TPL;
            if (PER * TPL == NB || j < NB) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[b][r] = line_base[(j + r * NB) * es];
            }
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int b = 0; b < PER; ++b) {
            int j = t + b * TPL;
            if (PER * TPL == NB || j < NB) {
                int k = (LS == 1) ? 0 : (j % LS);
                if (LS > 1) {
#pragma unroll
                    for (int r = 1; r < R; ++r) {
                        cplx<T> w = tw[r * k * (N / (LS * R))];
                        if (S > 0) w = conj(w);
                        v[b][r] = v[b][r] * w;
                    }
                }
                dftR<T, S, R>(v[b]);
                int o = (j - k) * R + k;
#pragma unroll
                for (int r = 0; r < R; ++r) line_base[(o + r * LS) * es] = v[b][r];
            }
        }
    }
    __syncthreads();
}

template <typename T, int N, int S, int TPL, int LS>
__device__ __forceinline__ void stockham_run(cplx<T>*, int, int, bool, const cplx<T>*, Radices<>) {}

template <typename T, int N, int S, int TPL, int LS, int R0, int... Rest>
__device__ __forceinline__ void stockham_run(cplx<T>* line_base, int es, int t, bool active, const cplx<T>* tw,
                                             Radices<R0, Rest...>) {
    stockham_pass<T, N, S, R0, LS, TPL>(line_base, es, t, active, tw);
    stockham_run<T, N, S, TPL, LS * R0>(line_base, es, t, active, tw, Radices<Rest...>{});
}

// FFT of `nlines` lines in LDS.  Lines start at buf + line * ls with
// element stride es.  LINES_FAST selects the lane mapping: consecutive lanes
// take consecutive lines (for element-strided, line-contiguous layouts) or
// consecutive elements of one line (for line-strided, element-contiguous
// layouts).  TPL threads work on one line (fewer than N / 8 give each thread
// several butterflies per pass).  All threads of the block must call this.
template <typename T, int N, int S, bool LINES_FAST, typename Plan = typename DefaultPlan<N>::type,
          int TPL = FFTShape<N>::TPL>
__device__ __forceinline__ void lds_fft_lines(cplx<T>* buf, int es, int ls, int nlines, const cplx<T>* tw) {
    const int conc = blockDim.x / TPL;
    const int tid = threadIdx.x;
    int ll, t;
    if (LINES_FAST) {
        ll = tid % conc;
        t = tid / conc;
    } else {
        ll = tid / TPL;
        t = tid % TPL;
    }
    for (int l0 = 0; l0 < nlines; l0 += conc) {
        int line = l0 + ll;
        bool active = (line < nlines) && (t < TPL) && (ll < conc);
        stockham_run<T, N, S, TPL, 1>(buf + (active ? line : 0) * ls, es, t, active, tw, Plan{});
    }
}

}  // namespace sdf
