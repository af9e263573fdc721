// Shared device-side helpers of the sdfdock kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sdf {

template <typename T>
struct __align__(2 * sizeof(T)) cplx {
    T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T r, T i) {
    cplx<T> c;
    c.re = r;
    c.im = i;
    return c;
}
template <typename T>
__device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
__device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
__device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
    return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__device__ __forceinline__ cplx<T> operator*(cplx<T> a, T s) { return mk(a.re * s, a.im * s); }
template <typename T>
__device__ __forceinline__ cplx<T> conj(cplx<T> a) { return mk(a.re, -a.im); }
// multiply by +i (s = +1) or -i (s = -1)
template <typename T, int S>
__device__ __forceinline__ cplx<T> mul_i(cplx<T> a) {
    return S > 0 ? mk(-a.im, a.re) : mk(a.im, -a.re);
}

// Cubic B-spline beta(s) and its derivative, piecewise cubic.
template <typename T>
__device__ __forceinline__ T bspline3(T s) {
    T a = s < T(0) ? -s : s;
    if (a < T(1)) return T(2) / T(3) - a * a + T(0.5) * a * a * a;
    if (a < T(2)) {
        T b = T(2) - a;
        return b * b * b * T(1.0 / 6.0);
    }
    return T(0);
}
// Weights of the 4 stencil nodes floor(y)-1+i, i = 0..3, at fractional part f in [0, 1).
template <typename T>
__device__ __forceinline__ void bspline3_weights(T f, T w[4]) {
    T g = T(1) - f;
    T f2 = f * f, f3 = f2 * f;
    w[0] = g * g * g * T(1.0 / 6.0);                       // beta(1 + f)
    w[1] = T(2) / T(3) - f2 + T(0.5) * f3;                 // beta(f)
    w[2] = T(2) / T(3) - g * g + T(0.5) * g * g * g;        // beta(1 - f)
    w[3] = f3 * T(1.0 / 6.0);                              // beta(2 - f)
}
// Six times the same 4 weights (callers fold the 1/6 into their scale).
template <typename T>
__device__ __forceinline__ void bspline3_weights6(T f, T w[4]) {
    const T g = T(1) - f;
    const T f2 = f * f, g2 = g * g;
    w[0] = g2 * g;                            // 6 beta(1 + f)
    w[1] = T(3) * f2 * f + (T(4) - T(6) * f2);  // 6 beta(f)
    w[2] = T(3) * g2 * g + (T(4) - T(6) * g2);  // 6 beta(1 - f)
    w[3] = f2 * f;                            // 6 beta(2 - f)
}
// d/dy of beta(node - y) for the same 4 nodes: -beta'(node - y).
template <typename T>
__device__ __forceinline__ void bspline3_dweights(T f, T d[4]) {
    T g = T(1) - f;
    d[0] = -T(0.5) * g * g;            // node - y = -(1 + f): -beta'(-(1+f)) = -(1/2)(1-f)^2
    d[1] = -T(2) * f + T(1.5) * f * f;  // node - y = -f
    d[2] = T(2) * g - T(1.5) * g * g;   // node - y = 1 - f
    d[3] = T(0.5) * f * f;              // node - y = 2 - f
}

// Load through a pointer known to address global memory (one fetched from a
// descriptor would otherwise become a flat access, which also occupies the
// LDS counter and so delays waits on LDS operations).
__device__ __forceinline__ cplx<float> gload(const cplx<float>* p, int64_t i) {
    using GPtr = const __attribute__((address_space(1))) unsigned long long*;
    const unsigned long long v = ((GPtr)p)[i];
    return mk(__uint_as_float(unsigned(v)), __uint_as_float(unsigned(v >> 32)));
}

// Raw buffer access through a gfx9 buffer descriptor of `bytes` bytes at
// `base` (the base must be wave-uniform).  A load whose offset lies at or past
// the end returns zeros and such a store is dropped, so an offset of
// kBufferNone reads zeros without a branch.  The descriptor is built in
// scalar registers; `soff` is a scalar offset added to the per-lane one.
constexpr uint32_t kBufferNone = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, int(bytes), 0x00020000);
}
__device__ __forceinline__ cplx<float> buffer_load_cf(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, int(voff), int(soff), 0);
    return mk(__uint_as_float(v[0]), __uint_as_float(v[1]));
}
__device__ __forceinline__ void buffer_store_cf(cplx<float> x, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                uint32_t soff) {
    using V2 = unsigned __attribute__((ext_vector_type(2)));
    V2 v;
    v[0] = __float_as_uint(x.re);
    v[1] = __float_as_uint(x.im);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, int(voff), int(soff), 0);
}
// a value the compiler may keep in a scalar register (it must be uniform)
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Pair-grouped column order (3D grids, N = 64 and 128).  Position p = 16 b + i
// holds kx = 8 b + i for i < 8 and kx = -(8 b + i - 8) mod N for i >= 8,
// except p = 8, which holds N / 2.  Every column's negative then sits in the
// same aligned block of 16 (at p ^ 8, or at p itself for kx = 0 and N / 2),
// so a pencil tile of row ky and its partner tile of row -ky cover the same
// aligned 128-byte segments.
template <int N>
__host__ __device__ __forceinline__ int col_pos(int kx) {
    if (kx == N / 2) return 8;
    if (kx < N / 2) return 16 * (kx >> 3) + (kx & 7);
    const int m = N - kx;
    return 16 * (m >> 3) + 8 + (m & 7);
}
template <int N>
__host__ __device__ __forceinline__ int col_kx(int p) {
    const int b = p >> 4, i = p & 15;
    if (i < 8) return 8 * b + i;
    if (p == 8) return N / 2;
    return N - (8 * b + i - 8);
}

// Column tiles (3D grids, N = 64 and 128): the spread slabs that K1 passes
// to K2, and the fixed spectrum K2 multiplies by, are stored as tiles of one
// row ky and one aligned block of 16 pair-grouped positions over every kz,
// kz-major, so the pencil pass reads each tile as one contiguous 16 N * 8
// bytes while K1 writes 128-byte pieces (HBM sustains scattered writes of
// that size far better than scattered reads).  Element (kz, ky, p) sits at
// ((ky (N / 16) + p / 16) N + kz) 16 + p % 16.
template <int N>
__host__ __device__ __forceinline__ int tile_index(int kz, int ky, int p) {
    return ((ky * (N / 16) + (p >> 4)) * N + kz) * 16 + (p & 15);
}

__device__ __forceinline__ int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

template <typename T>
__device__ __forceinline__ T dev_floor(T x);
template <>
__device__ __forceinline__ float dev_floor<float>(float x) { return floorf(x); }
template <>
__device__ __forceinline__ double dev_floor<double>(double x) { return floor(x); }

}  // namespace sdf
