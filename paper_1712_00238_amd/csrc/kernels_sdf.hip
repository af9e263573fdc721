// Skeletal density function on a grid (eq. 10A, 11, 12a, 13, 15, 16c, 17t).
//
// One thread per grid node, boundary samples streamed through LDS in tiles
// that every thread of the block reads by broadcast.  Pass 1 finds the
// nearest sample (signed distance and membership); pass 2 sums the kernel
// over the samples inside the eps-approximate contact ball.  With
// r = eta / |xi| the kernel of eq. 15 on zeta = xi + i eta reduces to
//   phi = lambda / (2 pi sigma xi^2) * G(r) * P(r) / (1 + r^2)^2,
//   G = exp(-(r - 1)^2 / (2 sigma^2)),  P = (1 - i r)^2 outside, (1 + i r)^2 inside,
// so a pair costs one reciprocal square root, one exponential and one
// reciprocal, with no trigonometric calls.
#include "common.hpp"
#include "launch.hpp"

namespace sdf {

namespace {

constexpr int kSdfBlock = 256;
constexpr int kSdfTile = 256;

template <typename T>
struct __align__(4 * sizeof(T)) v4 {
    T x, y, z, w;
};

template <typename T>
__device__ __forceinline__ T fast_rsqrt(T x);
template <>
__device__ __forceinline__ float fast_rsqrt<float>(float x) { return rsqrtf(x); }
template <>
__device__ __forceinline__ double fast_rsqrt<double>(double x) { return rsqrt(x); }

template <typename T>
__device__ __forceinline__ T dev_exp(T x);
template <>
__device__ __forceinline__ float dev_exp<float>(float x) { return expf(x); }
template <>
__device__ __forceinline__ double dev_exp<double>(double x) { return exp(x); }

template <typename T>
__global__ __launch_bounds__(kSdfBlock) void sdf_build_kernel(const T* __restrict__ q, const T* __restrict__ nrm,
                                                              const T* __restrict__ w, int64_t ns, GridDesc g,
                                                              ParamDesc prm, cplx<T>* __restrict__ out,
                                                              int64_t nnodes) {
    __shared__ v4<T> sq[kSdfTile];  // (qx, qy, qz, w)
    __shared__ v4<T> sn[kSdfTile];  // (nx, ny, nz, 0)

    const int64_t node = int64_t(blockIdx.x) * kSdfBlock + threadIdx.x;
    const bool valid = node < nnodes;
    const int64_t nn = valid ? node : 0;
    const int i = int(nn % g.nx);
    const int j = int((nn / g.nx) % g.ny);
    const int k = int(nn / (int64_t(g.nx) * g.ny));
    const T px = T(g.ox + g.h * i), py = T(g.oy + g.h * j), pz = T(g.oz + g.h * k);

    // ---- pass 1: nearest sample, lowest index on exact ties
    T best = T(INFINITY);
    int64_t jbest = 0;
    for (int64_t t0 = 0; t0 < ns; t0 += kSdfTile) {
        const int cnt = int(ns - t0 < kSdfTile ? ns - t0 : kSdfTile);
        __syncthreads();
        for (int a = threadIdx.x; a < cnt; a += kSdfBlock) {
            const int64_t s = t0 + a;
            sq[a] = v4<T>{q[3 * s], q[3 * s + 1], q[3 * s + 2], w[s]};
        }
        __syncthreads();
#pragma unroll 8
        for (int a = 0; a < cnt; ++a) {
            const v4<T> s = sq[a];
            const T dx = px - s.x, dy = py - s.y, dz = pz - s.z;
            const T d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < best) {
                best = d2;
                jbest = t0 + a;
            }
        }
    }
    const T qx = q[3 * jbest], qy = q[3 * jbest + 1], qz = q[3 * jbest + 2];
    const T dot = (px - qx) * nrm[3 * jbest] + (py - qy) * nrm[3 * jbest + 1] + (pz - qz) * nrm[3 * jbest + 2];
    const int pmc = dot > T(0) ? 1 : (dot < T(0) ? -1 : 0);
    const T xi2 = best;
    const T xi_abs = sqrt(xi2);
    const bool live = valid && pmc != 0 && xi_abs >= T(prm.xi_floor);

    // ---- pass 2: truncated kernel sum over the contact ball
    const T radius = T(1.0 + prm.eps) * xi_abs;
    const T r2max = radius * radius;
    const T inv_xi = T(1) / xi_abs;
    const T inv2s2 = T(0.5 / (prm.sigma * prm.sigma));
    const T im_sign = pmc > 0 ? T(-2) : T(2);  // P = (1 - r^2) -+ 2 i r
    T acc_re = T(0), acc_im = T(0);
    // a block whose nodes are all dead still runs the loop for its barriers
    for (int64_t t0 = 0; t0 < ns; t0 += kSdfTile) {
        const int cnt = int(ns - t0 < kSdfTile ? ns - t0 : kSdfTile);
        __syncthreads();
        for (int a = threadIdx.x; a < cnt; a += kSdfBlock) {
            const int64_t s = t0 + a;
            sq[a] = v4<T>{q[3 * s], q[3 * s + 1], q[3 * s + 2], w[s]};
            sn[a] = v4<T>{nrm[3 * s], nrm[3 * s + 1], nrm[3 * s + 2], T(0)};
        }
        __syncthreads();
        if (live) {
#pragma unroll 4
            for (int a = 0; a < cnt; ++a) {
                const v4<T> s = sq[a];
                const T dx = px - s.x, dy = py - s.y, dz = pz - s.z;
                const T d2 = dx * dx + dy * dy + dz * dz;
                if (d2 <= r2max) {
                    const v4<T> nv = sn[a];
                    const T inv_eta = fast_rsqrt(d2);
                    const T eta = d2 * inv_eta;
                    const T r = eta * inv_xi;
                    const T cos_t = (dx * nv.x + dy * nv.y + dz * nv.z) * inv_eta;
                    const T x = r - T(1);
                    const T G = dev_exp(-x * x * inv2s2);
                    const T rr = r * r;
                    const T den = T(1) + rr;
                    const T coef = s.w * cos_t * G / (den * den);
                    acc_re += coef * (T(1) - rr);
                    acc_im += coef * (im_sign * r);
                }
            }
        }
    }
    if (valid) {
        cplx<T> res = mk(T(0), T(0));
        if (live) {
            const T lam = pmc > 0 ? T(prm.lambda1) : T(-prm.lambda2);
            const T scale = lam / (T(2.0 * 3.14159265358979323846 * prm.sigma) * xi2);
            res = mk(acc_re * scale, acc_im * scale);
        }
        out[node] = res;
    }
}

}  // namespace

template <typename T>
hipError_t launch_sdf_build(const T* q, const T* n, const T* w, int64_t ns, const GridDesc& g, const ParamDesc& p,
                            void* rho_out, hipStream_t s) {
    const int64_t nnodes = int64_t(g.nx) * g.ny * g.nz;
    const int64_t blocks = (nnodes + kSdfBlock - 1) / kSdfBlock;
    hipLaunchKernelGGL(sdf_build_kernel<T>, dim3(unsigned(blocks)), dim3(kSdfBlock), 0, s, q, n, w, ns, g, p,
                       static_cast<cplx<T>*>(rho_out), nnodes);
    return hipGetLastError();
}

template hipError_t launch_sdf_build<float>(const float*, const float*, const float*, int64_t, const GridDesc&,
                                            const ParamDesc&, void*, hipStream_t);
template hipError_t launch_sdf_build<double>(const double*, const double*, const double*, int64_t, const GridDesc&,
                                             const ParamDesc&, void*, hipStream_t);

}  // namespace sdf
