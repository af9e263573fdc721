// Nonequispaced route of the search (Implementation section): octree-
// adaptive samples of the moving affinity, and per rotation the type-1
// nonequispaced transform of the rotated samples by "exponential of
// semicircle" spreading on the 2x oversampled grid, FFT, crop and
// deconvolution (Barnett, Magland and af Klinteberg, 2019), followed by the
// spectral product with the fixed part.
//
// Octree reading: cells of 2^l nodes per side (l <= max_level <= 3, aligned
// to multiples of 2^l) whose coefficient spread (max - min of Re and of Im)
// is below tol * A, A = max_k max(|Re c_k|, |Im c_k|), become one leaf at
// the cell centre carrying the sum of the cell's coefficients; each node
// goes to the highest such cell above it, or stays a leaf of its own.
// Leaves whose nodes are all zero are dropped.  Leaves are emitted per
// 8^3 (planar 8^2) block in flat block order, Morton order within a block.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include "common.hpp"
#include "launch.hpp"

namespace sdf {
namespace {

template <typename T>
struct UBits;
template <>
struct UBits<float> {
    using U = unsigned int;
};
template <>
struct UBits<double> {
    using U = unsigned long long;
};

__device__ __forceinline__ float from_bits(unsigned int u) { return __uint_as_float(u); }
__device__ __forceinline__ double from_bits(unsigned long long u) { return __longlong_as_double((long long)u); }
__device__ __forceinline__ unsigned int to_bits(float v) { return __float_as_uint(v); }
__device__ __forceinline__ unsigned long long to_bits(double v) {
    return (unsigned long long)__double_as_longlong(v);
}

__device__ __forceinline__ float dmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double dmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float dmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double dmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float dabs(float a) { return fabsf(a); }
__device__ __forceinline__ double dabs(double a) { return fabs(a); }
__device__ __forceinline__ float dceil(float a) { return ceilf(a); }
__device__ __forceinline__ double dceil(double a) { return ceil(a); }
__device__ __forceinline__ float dexp(float a) { return expf(a); }
__device__ __forceinline__ double dexp(double a) { return exp(a); }
__device__ __forceinline__ float dsqrt(float a) { return sqrtf(a); }
__device__ __forceinline__ double dsqrt(double a) { return sqrt(a); }

// ------------------------------------------------------------------ octree
template <typename U>
__global__ void clear_bits_kernel(U* p) {
    if (threadIdx.x == 0) p[0] = U(0);
}

// A as the bit pattern of a non-negative value: integer max orders such
// patterns like the values, so the result is exact and order-independent.
template <typename T>
__global__ __launch_bounds__(256) void absmax_kernel(const cplx<T>* __restrict__ c, int64_t n,
                                                     typename UBits<T>::U* __restrict__ out) {
    T m = T(0);
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        const cplx<T> v = c[i];
        m = dmax(m, dmax(dabs(v.re), dabs(v.im)));
    }
    for (int off = 32; off > 0; off >>= 1) m = dmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0 && m > T(0)) atomicMax(out, to_bits(m));
}

constexpr int kOctBlock = 512;

// One block per 8^DIM node block, thread t = Morton index (x bit lowest).
// Level-l cells are runs of 2^(DIM l) consecutive threads, reduced with
// butterflies inside a wave and through LDS across the 8 waves (3D, l = 3).
// EMIT = false counts the block's leaves; EMIT = true writes them at
// offsets[block] + (leaves of lower threads).
template <typename T, int DIM, bool EMIT>
__global__ __launch_bounds__(kOctBlock) void octree_kernel(const cplx<T>* __restrict__ c, int nm,
                                                           const typename UBits<T>::U* __restrict__ amax, T tol,
                                                           int max_level, int* __restrict__ counts,
                                                           const int* __restrict__ offsets, T* __restrict__ pos,
                                                           cplx<T>* __restrict__ out_c, int* __restrict__ out_level) {
    constexpr int NT = DIM == 3 ? 512 : 64;
    constexpr int NW = NT / 64;
    __shared__ T s_mnr[NW], s_mxr[NW], s_mni[NW], s_mxi[NW];
    __shared__ double s_sr[NW], s_si[NW];
    __shared__ int s_nz[NW], s_cnt[NW];
    const int t = int(threadIdx.x), lane = t & 63, wq = t >> 6;
    int lx = 0, ly = 0, lz = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        lx |= ((t >> (DIM * b)) & 1) << b;
        ly |= ((t >> (DIM * b + 1)) & 1) << b;
        if (DIM == 3) lz |= ((t >> (DIM * b + 2)) & 1) << b;
    }
    const unsigned nb = unsigned(nm >> 3);
    const int bx = int(blockIdx.x % nb), by = int((blockIdx.x / nb) % nb);
    const int bz = DIM == 3 ? int(blockIdx.x / (nb * nb)) : 0;
    const int i = bx * 8 + lx, j = by * 8 + ly, k = bz * 8 + lz;
    const cplx<T> v = c[(int64_t(k) * nm + j) * nm + i];
    const T tau = tol * from_bits(amax[0]);

    T mnr = v.re, mxr = v.re, mni = v.im, mxi = v.im;
    double sr = double(v.re), si = double(v.im);
    int nz = (v.re != T(0) || v.im != T(0)) ? 1 : 0;
    // the leaf this node belongs to: its level and the cell's sums
    int lv = 0;
    double csr = sr, csi = si;
    int cnz = nz;
#pragma unroll
    for (int l = 1; l <= 3; ++l) {
#pragma unroll
        for (int b = DIM * (l - 1); b < DIM * l; ++b) {
            if (b < 6) {
                const int off = 1 << b;
                mnr = dmin(mnr, __shfl_xor(mnr, off));
                mxr = dmax(mxr, __shfl_xor(mxr, off));
                mni = dmin(mni, __shfl_xor(mni, off));
                mxi = dmax(mxi, __shfl_xor(mxi, off));
                sr += __shfl_xor(sr, off);
                si += __shfl_xor(si, off);
                nz |= __shfl_xor(nz, off);
            }
        }
        if (DIM * l > 6) {
            // every lane holds its wave's values; combine the waves in order
            if (lane == 0) {
                s_mnr[wq] = mnr;
                s_mxr[wq] = mxr;
                s_mni[wq] = mni;
                s_mxi[wq] = mxi;
                s_sr[wq] = sr;
                s_si[wq] = si;
                s_nz[wq] = nz;
            }
            __syncthreads();
            mnr = s_mnr[0];
            mxr = s_mxr[0];
            mni = s_mni[0];
            mxi = s_mxi[0];
            sr = s_sr[0];
            si = s_si[0];
            nz = s_nz[0];
#pragma unroll
            for (int w = 1; w < NW; ++w) {
                mnr = dmin(mnr, s_mnr[w]);
                mxr = dmax(mxr, s_mxr[w]);
                mni = dmin(mni, s_mni[w]);
                mxi = dmax(mxi, s_mxi[w]);
                sr += s_sr[w];
                si += s_si[w];
                nz |= s_nz[w];
            }
        }
        // spreads only grow with the cell, so the flat levels <= max_level
        // run from 1 up to some level; the last one is the leaf
        if (l <= max_level && (mxr - mnr < tau) && (mxi - mni < tau)) {
            lv = l;
            csr = sr;
            csi = si;
            cnz = nz;
        }
    }
    const bool keep = ((t & ((1 << (DIM * lv)) - 1)) == 0) && cnz != 0;
    const unsigned long long bal = __ballot(keep);
    if (lane == 0) s_cnt[wq] = __popcll(bal);
    __syncthreads();
    if (!EMIT) {
        if (t == 0) {
            int tot = 0;
            for (int w = 0; w < NW; ++w) tot += s_cnt[w];
            counts[blockIdx.x] = tot;
        }
        return;
    }
    if (!keep) return;
    int at = offsets[blockIdx.x];
    for (int w = 0; w < wq; ++w) at += s_cnt[w];
    at += __popcll(bal & ((1ull << lane) - 1ull));
    const T hs = T(0.5) * T((1 << lv) - 1), hm = T(0.5) * T(nm);
    pos[3 * int64_t(at)] = T(i) + hs - hm;
    pos[3 * int64_t(at) + 1] = T(j) + hs - hm;
    pos[3 * int64_t(at) + 2] = DIM == 3 ? T(k) + hs - hm : T(0);
    out_c[at] = mk(T(csr), T(csi));
    if (out_level) out_level[at] = lv;
}

__global__ void octree_total_kernel(const int* __restrict__ counts, const int* __restrict__ offsets, int nblk,
                                    int64_t* __restrict__ out) {
    if (threadIdx.x == 0) out[0] = int64_t(offsets[nblk - 1]) + counts[nblk - 1];
}

// ------------------------------------------------------------------ type-1 transform
constexpr double kEsBetaPerWidth = 2.30;  // beta = 2.30 w at oversampling 2
constexpr int kEsQuad = 4096;

// inv[j] = 1 / phihat(kappa_j), kappa_j = j (j < N/2) or j - N, with
// phihat(kappa) = int phi(2x/w) cos(2 pi kappa x / (2N)) dx over |x| <= w/2.
// With 2x/w = sin(theta) the integrand exp(beta (cos theta - 1))
// cos(pi kappa w sin(theta) / (2N)) (w/2) cos(theta) is smooth on
// [-pi/2, pi/2] (the square-root edge of phi is gone), so composite Simpson
// in FP64 converges fast even for narrow kernels, whose edge value e^-beta
// is not small.
template <typename T>
__global__ void es_deconv_kernel(int N, int w, T* __restrict__ inv) {
    const int jj = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (jj >= N) return;
    const double kap = jj < N / 2 ? double(jj) : double(jj - N);
    const double beta = kEsBetaPerWidth * w, half = 0.5 * w, h = M_PI / kEsQuad;
    double acc = 0.0;
    for (int q = 1; q < kEsQuad; ++q) {  // the end points contribute cos(+-pi/2) = 0
        const double th = -0.5 * M_PI + q * h;
        double st, ct;
        sincos(th, &st, &ct);
        const double g = exp(beta * (ct - 1.0)) * cospi(kap * half * st / double(N)) * half * ct;
        acc += (q & 1 ? 4.0 : 2.0) * g;
    }
    inv[jj] = T(1.0 / (acc * h / 3.0));
}

// One thread per sample and rotation: the reflected rotated position
// -R x_k, doubled onto the fine grid of nf = 2N nodes (periodic), spread
// over W^DIM nodes with global atomics.  `fine` must be zero.
template <typename T, int DIM, int W>
__global__ __launch_bounds__(256) void nfft_spread_kernel(const T* __restrict__ pos, const cplx<T>* __restrict__ c,
                                                          int64_t m, const T* __restrict__ R, int nf,
                                                          cplx<T>* __restrict__ fine) {
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k >= m) return;
    const cplx<T> ck = c[k];
    if (ck.re == T(0) && ck.im == T(0)) return;
    const T* r = R + 9 * blockIdx.y;
    const T px = pos[3 * k], py = pos[3 * k + 1], pz = DIM == 3 ? pos[3 * k + 2] : T(0);
    const int64_t gsz = DIM == 3 ? int64_t(nf) * nf * nf : int64_t(nf) * nf;
    cplx<T>* g = fine + int64_t(blockIdx.y) * gsz;
    const T beta = T(kEsBetaPerWidth * W), half = T(0.5 * W), zs = T(2.0 / W), fn = T(nf);
    int l0[3] = {0, 0, 0};
    T wt[3][W];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        T y = -T(2) * (r[3 * a] * px + r[3 * a + 1] * py + r[3 * a + 2] * pz);
        y = y - dev_floor(y / fn) * fn;
        l0[a] = int(dceil(y - half));
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const T z = (T(l0[a] + q) - y) * zs;
            const T s = T(1) - z * z;
            wt[a][q] = s >= T(0) ? dexp(beta * (dsqrt(s) - T(1))) : T(0);
        }
    }
    if (DIM == 2) {
#pragma unroll
        for (int b = 0; b < W; ++b) {
            const int yy = wrap(l0[1] + b, nf);
#pragma unroll
            for (int a = 0; a < W; ++a) {
                const T wgt = wt[0][a] * wt[1][b];
                cplx<T>* p = g + int64_t(yy) * nf + wrap(l0[0] + a, nf);
                atomicAdd(&p->re, ck.re * wgt);
                atomicAdd(&p->im, ck.im * wgt);
            }
        }
        return;
    }
#pragma unroll
    for (int cz = 0; cz < W; ++cz) {
        const int zz = wrap(l0[2] + cz, nf);
#pragma unroll
        for (int b = 0; b < W; ++b) {
            const int yy = wrap(l0[1] + b, nf);
            const T wyz = wt[1][b] * wt[2][cz];
            cplx<T>* row = g + (int64_t(zz) * nf + yy) * nf;
#pragma unroll
            for (int a = 0; a < W; ++a) {
                const T wgt = wt[0][a] * wyz;
                cplx<T>* p = row + wrap(l0[0] + a, nf);
                atomicAdd(&p->re, ck.re * wgt);
                atomicAdd(&p->im, ck.im * wgt);
            }
        }
    }
}

// The N^d central modes of the fine transform, deconvolved and multiplied by
// the fixed part's spectrum: out[b][j] = G[b][j mod-shifted] inv inv inv spec[j].
template <typename T>
__global__ void nfft_crop_kernel(const cplx<T>* __restrict__ fine, int N, int planar, int batch,
                                 const T* __restrict__ inv, const cplx<T>* __restrict__ spec,
                                 cplx<T>* __restrict__ out) {
    const int nf = 2 * N;
    const int64_t G = planar ? int64_t(N) * N : int64_t(N) * N * N;
    const int64_t Gf = planar ? int64_t(nf) * nf : int64_t(nf) * nf * nf;
    const int64_t total = G * batch;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t b = e / G, idx = e - b * G;
        const int jx = int(idx % N), jy = int((idx / N) % N), jz = planar ? 0 : int(idx / (int64_t(N) * N));
        const int fx = jx < N / 2 ? jx : jx + N, fy = jy < N / 2 ? jy : jy + N;
        const int fz = planar ? 0 : (jz < N / 2 ? jz : jz + N);
        const T sc = inv[jx] * inv[jy] * (planar ? T(1) : inv[jz]);
        out[e] = fine[b * Gf + (int64_t(fz) * nf + fy) * nf + fx] * sc * spec[idx];
    }
}

template <typename T, int DIM>
hipError_t spread_width(const T* pos, const cplx<T>* c, int64_t m, const T* R, int batch, int nf, int w,
                        cplx<T>* fine, hipStream_t s) {
    const dim3 grid(unsigned((m + 255) / 256), unsigned(batch));
    switch (w) {
#define SDF_NFFT_W(WW)                                                                                          \
    case WW:                                                                                                    \
        hipLaunchKernelGGL((nfft_spread_kernel<T, DIM, WW>), grid, dim3(256), 0, s, pos, c, m, R, nf, fine); \
        break;
        SDF_NFFT_W(2)
        SDF_NFFT_W(3)
        SDF_NFFT_W(4)
        SDF_NFFT_W(5)
        SDF_NFFT_W(6)
        SDF_NFFT_W(7)
        SDF_NFFT_W(8)
#undef SDF_NFFT_W
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// workspace of launch_octree: coefficients, A, per-block counts and
// offsets, scan temporaries
struct OctWs {
    size_t coef, amax, counts, offsets, temp, temp_bytes, total;
};

size_t al256(size_t v) { return (v + 255) / 256 * 256; }

OctWs oct_ws_layout(int nm, bool planar, size_t elem) {
    const int64_t K = planar ? int64_t(nm) * nm : int64_t(nm) * nm * nm;
    const int nblk = int(K / (planar ? 64 : 512));
    size_t temp_bytes = 0;
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, temp_bytes, static_cast<const int*>(nullptr),
                                           static_cast<int*>(nullptr), nblk);
    OctWs L{};
    size_t off = 0;
    L.coef = off;
    off += al256(2 * elem * size_t(K));
    L.amax = off;
    off += 256;
    L.counts = off;
    off += al256(sizeof(int) * size_t(nblk));
    L.offsets = off;
    off += al256(sizeof(int) * size_t(nblk));
    L.temp = off;
    L.temp_bytes = temp_bytes;
    off += al256(temp_bytes);
    L.total = off;
    return L;
}

}  // namespace

size_t octree_workspace_bytes(int nm, bool planar, size_t elem) { return oct_ws_layout(nm, planar, elem).total; }

template <typename T>
hipError_t launch_octree(const void* rho_m, const T* w_m, int nm, bool planar, double tol, int max_level, T* pos,
                         void* c_out, int* level, int64_t* count_out, void* ws, hipStream_t s) {
    using U = typename UBits<T>::U;
    const OctWs L = oct_ws_layout(nm, planar, sizeof(T));
    char* base = static_cast<char*>(ws);
    const int64_t K = planar ? int64_t(nm) * nm : int64_t(nm) * nm * nm;
    const int nblk = int(K / (planar ? 64 : 512));
    cplx<T>* coef = reinterpret_cast<cplx<T>*>(base + L.coef);
    U* amax = reinterpret_cast<U*>(base + L.amax);
    int* counts = reinterpret_cast<int*>(base + L.counts);
    int* offsets = reinterpret_cast<int*>(base + L.offsets);
    hipError_t e = launch_coef<T>(rho_m, w_m, K, coef, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((clear_bits_kernel<U>), dim3(1), dim3(64), 0, s, amax);
    const int64_t ab = (K + 255) / 256;
    hipLaunchKernelGGL((absmax_kernel<T>), dim3(unsigned(ab < 2048 ? ab : 2048)), dim3(256), 0, s, coef, K, amax);
    const T tl = T(tol);
    cplx<T>* oc = static_cast<cplx<T>*>(c_out);
    if (planar) {
        hipLaunchKernelGGL((octree_kernel<T, 2, false>), dim3(nblk), dim3(64), 0, s, coef, nm, amax, tl, max_level,
                           counts, offsets, pos, oc, level);
    } else {
        hipLaunchKernelGGL((octree_kernel<T, 3, false>), dim3(nblk), dim3(512), 0, s, coef, nm, amax, tl, max_level,
                           counts, offsets, pos, oc, level);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t tb = L.temp_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(base + L.temp, tb, counts, offsets, nblk, s);
    if (e != hipSuccess) return e;
    if (planar) {
        hipLaunchKernelGGL((octree_kernel<T, 2, true>), dim3(nblk), dim3(64), 0, s, coef, nm, amax, tl, max_level,
                           counts, offsets, pos, oc, level);
    } else {
        hipLaunchKernelGGL((octree_kernel<T, 3, true>), dim3(nblk), dim3(512), 0, s, coef, nm, amax, tl, max_level,
                           counts, offsets, pos, oc, level);
    }
    hipLaunchKernelGGL(octree_total_kernel, dim3(1), dim3(64), 0, s, counts, offsets, nblk, count_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_es_deconv(int N, int w, T* inv, hipStream_t s) {
    hipLaunchKernelGGL((es_deconv_kernel<T>), dim3(unsigned((N + 63) / 64)), dim3(64), 0, s, N, w, inv);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_nfft_modes(const T* pos, const void* c, int64_t m, const T* R, int batch, int N, bool planar,
                             int w, const T* inv, const void* spec, void* fine, void* out, hipStream_t s) {
    const int nf = 2 * N;
    const int64_t Gf = planar ? int64_t(nf) * nf : int64_t(nf) * nf * nf;
    const int64_t G = planar ? int64_t(N) * N : int64_t(N) * N * N;
    hipError_t e = launch_zero<T>(fine, Gf * batch, s);
    if (e != hipSuccess) return e;
    const cplx<T>* cc = static_cast<const cplx<T>*>(c);
    cplx<T>* fg = static_cast<cplx<T>*>(fine);
    if (m > 0) {
        e = planar ? spread_width<T, 2>(pos, cc, m, R, batch, nf, w, fg, s)
                   : spread_width<T, 3>(pos, cc, m, R, batch, nf, w, fg, s);
        if (e != hipSuccess) return e;
    }
    e = launch_fft3<T>(fine, nf, planar, batch, -1, 1.0, s);
    if (e != hipSuccess) return e;
    const int64_t cb = (G * batch + 255) / 256;
    hipLaunchKernelGGL((nfft_crop_kernel<T>), dim3(unsigned(cb < 16384 ? cb : 16384)), dim3(256), 0, s, fg, N,
                       planar ? 1 : 0, batch, inv, static_cast<const cplx<T>*>(spec), static_cast<cplx<T>*>(out));
    return hipGetLastError();
}

template hipError_t launch_octree<float>(const void*, const float*, int, bool, double, int, float*, void*, int*,
                                         int64_t*, void*, hipStream_t);
template hipError_t launch_octree<double>(const void*, const double*, int, bool, double, int, double*, void*, int*,
                                          int64_t*, void*, hipStream_t);
template hipError_t launch_es_deconv<float>(int, int, float*, hipStream_t);
template hipError_t launch_es_deconv<double>(int, int, double*, hipStream_t);
template hipError_t launch_nfft_modes<float>(const float*, const void*, int64_t, const float*, int, int, bool, int,
                                             const float*, const void*, void*, void*, hipStream_t);
template hipError_t launch_nfft_modes<double>(const double*, const void*, int64_t, const double*, int, int, bool,
                                              int, const double*, const void*, void*, void*, hipStream_t);

}  // namespace sdf
