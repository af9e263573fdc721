// Skeletal density function on a grid (eq. 10A, 11, 12a, 13, 15, 16c, 17t).
//
// One thread per grid node; a block covers a compact 8 x 8 x 4 brick of
// nodes (16 x 16 in the plane) so that positions relative to the brick's
// corner are small.  Boundary samples stream through LDS in tiles that every
// thread reads by broadcast.
//
// Pass 1 finds the nearest sample, its membership sign and the distance
// floor test.  These are discrete decisions, taken in FP64 from FP64 sample
// positions in both precisions, so the classification of every node is the
// one an FP64 evaluation makes.
//
// Pass 2 sums the kernel over the samples inside the eps-approximate contact
// ball, in the context's precision T, on brick-relative coordinates.  A
// sample whose squared distance lies within 1e-4 (relative) of the ball's
// squared radius is re-tested in FP64.
//
// With r = eta / |xi| the kernel of eq. 15 on zeta = xi + i eta reduces to
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

// FP32 uses the hardware approximations directly (about 1 ulp each):
// v_rsq_f32 (live pairs have d^2 >= xi_floor^2, far from denormals),
// v_exp_f32 on a base-2 argument of magnitude below about 7, and v_rcp_f32.
// FP64 uses the correctly rounded library functions.
template <typename T>
__device__ __forceinline__ T fast_rsqrt(T x);
template <>
__device__ __forceinline__ float fast_rsqrt<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <>
__device__ __forceinline__ double fast_rsqrt<double>(double x) { return rsqrt(x); }

template <typename T>
__device__ __forceinline__ T dev_exp2(T x);
template <>
__device__ __forceinline__ float dev_exp2<float>(float x) { return __builtin_amdgcn_exp2f(x); }
template <>
__device__ __forceinline__ double dev_exp2<double>(double x) { return exp2(x); }

template <typename T>
__device__ __forceinline__ T dev_rcp(T x);
template <>
__device__ __forceinline__ float dev_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ __forceinline__ double dev_rcp<double>(double x) { return 1.0 / x; }

// brick of nodes handled by one block
struct Brick {
    int bx, by, bz;
};
__host__ __device__ inline Brick brick_shape(int nz) { return nz == 1 ? Brick{16, 16, 1} : Brick{8, 8, 4}; }

template <typename T>
__global__ __launch_bounds__(kSdfBlock) void sdf_build_kernel(const double* __restrict__ q,
                                                              const double* __restrict__ nrm,
                                                              const double* __restrict__ w, int64_t ns, GridDesc g,
                                                              ParamDesc prm, cplx<T>* __restrict__ out) {
    __shared__ v4<double> sq[2 * kSdfTile];  // pass 1: (qx, qy, qz, -); pass 2: reused as two T tiles
    v4<T>* sq2 = reinterpret_cast<v4<T>*>(sq);             // (qx, qy, qz, w) relative to the brick
    v4<T>* sn2 = reinterpret_cast<v4<T>*>(sq) + kSdfTile;  // (nx, ny, nz, 0)

    const Brick br = brick_shape(g.nz);
    const int nbx = (g.nx + br.bx - 1) / br.bx, nby = (g.ny + br.by - 1) / br.by;
    const int blk = blockIdx.x;
    const int i0 = (blk % nbx) * br.bx, j0 = ((blk / nbx) % nby) * br.by, k0 = (blk / (nbx * nby)) * br.bz;
    const int li = threadIdx.x % br.bx, lj = (threadIdx.x / br.bx) % br.by, lk = threadIdx.x / (br.bx * br.by);
    const int i = i0 + li, j = j0 + lj, k = k0 + lk;
    const bool valid = i < g.nx && j < g.ny && k < g.nz;
    // brick corner (FP64) and this node relative to it
    const double cx = g.ox + g.h * i0, cy = g.oy + g.h * j0, cz = g.oz + g.h * k0;
    const double rx = g.h * li, ry = g.h * lj, rz = g.h * lk;
    const double px = cx + rx, py = cy + ry, pz = cz + rz;

    // ---- pass 1 (FP64): nearest sample, lowest index on exact ties
    double best = INFINITY;
    int64_t jbest = 0;
    for (int64_t t0 = 0; t0 < ns; t0 += kSdfTile) {
        const int cnt = int(ns - t0 < kSdfTile ? ns - t0 : kSdfTile);
        __syncthreads();
        for (int a = threadIdx.x; a < cnt; a += kSdfBlock) {
            const int64_t s = t0 + a;
            sq[a] = v4<double>{q[3 * s], q[3 * s + 1], q[3 * s + 2], 0.0};
        }
        __syncthreads();
#pragma unroll 4
        for (int a = 0; a < cnt; ++a) {
            const v4<double> s = sq[a];
            const double dx = px - s.x, dy = py - s.y, dz = pz - s.z;
            const double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < best) {
                best = d2;
                jbest = t0 + a;
            }
        }
    }
    const double dot = (px - q[3 * jbest]) * nrm[3 * jbest] + (py - q[3 * jbest + 1]) * nrm[3 * jbest + 1] +
                       (pz - q[3 * jbest + 2]) * nrm[3 * jbest + 2];
    const int pmc = dot > 0.0 ? 1 : (dot < 0.0 ? -1 : 0);
    const double xi_abs64 = sqrt(best);
    const bool live = valid && pmc != 0 && xi_abs64 >= prm.xi_floor;

    // ---- pass 2 (T): truncated kernel sum over the contact ball
    const double r2max64 = (1.0 + prm.eps) * (1.0 + prm.eps) * best;
    const T r2lo = T(r2max64 * (1.0 - 1e-4)), r2hi = T(r2max64 * (1.0 + 1e-4));
    const T xi_abs = T(xi_abs64);
    const T inv_xi = T(1.0 / xi_abs64);
    // exp(-x^2 / (2 sigma^2)) = 2^(-x^2 log2(e) / (2 sigma^2))
    const T inv2s2 = T(0.5 * 1.4426950408889634 / (prm.sigma * prm.sigma));
    const T im_sign = pmc > 0 ? T(-2) : T(2);  // P = (1 - r^2) -+ 2 i r
    const T prx = T(rx), pry = T(ry), prz = T(rz);
    T acc_re = T(0), acc_im = T(0);
    (void)xi_abs;
    // a block whose nodes are all dead still runs the loop for its barriers
    for (int64_t t0 = 0; t0 < ns; t0 += kSdfTile) {
        const int cnt = int(ns - t0 < kSdfTile ? ns - t0 : kSdfTile);
        __syncthreads();
        for (int a = threadIdx.x; a < cnt; a += kSdfBlock) {
            const int64_t s = t0 + a;
            sq2[a] = v4<T>{T(q[3 * s] - cx), T(q[3 * s + 1] - cy), T(q[3 * s + 2] - cz), T(w[s])};
            sn2[a] = v4<T>{T(nrm[3 * s]), T(nrm[3 * s + 1]), T(nrm[3 * s + 2]), T(0)};
        }
        __syncthreads();
        if (live) {
#pragma unroll 4
            for (int a = 0; a < cnt; ++a) {
                const v4<T> s = sq2[a];
                const T dx = prx - s.x, dy = pry - s.y, dz = prz - s.z;
                const T d2 = dx * dx + dy * dy + dz * dz;
                bool in = d2 <= r2lo;
                if (!in && d2 <= r2hi) {  // near the sphere: decide in FP64
                    const int64_t sj = t0 + a;
                    const double ex = px - q[3 * sj], ey = py - q[3 * sj + 1], ez = pz - q[3 * sj + 2];
                    in = ex * ex + ey * ey + ez * ez <= r2max64;
                }
                if (in) {
                    const v4<T> nv = sn2[a];
                    const T inv_eta = fast_rsqrt(d2);
                    const T eta = d2 * inv_eta;
                    const T r = eta * inv_xi;
                    const T cos_t = (dx * nv.x + dy * nv.y + dz * nv.z) * inv_eta;
                    const T x = r - T(1);
                    const T G = dev_exp2(-x * x * inv2s2);
                    const T rr = r * r;
                    const T den = T(1) + rr;
                    const T coef = s.w * cos_t * G * dev_rcp(den * den);
                    acc_re += coef * (T(1) - rr);
                    acc_im += coef * (im_sign * r);
                }
            }
        }
    }
    if (valid) {
        cplx<T> res = mk(T(0), T(0));
        if (live) {
            const double lam = pmc > 0 ? prm.lambda1 : -prm.lambda2;
            const T scale = T(lam / (2.0 * 3.14159265358979323846 * prm.sigma * best));
            res = mk(acc_re * scale, acc_im * scale);
        }
        out[(int64_t(k) * g.ny + j) * g.nx + i] = res;
    }
}

}  // namespace

template <typename T>
hipError_t launch_sdf_build(const double* q, const double* n, const double* w, int64_t ns, const GridDesc& g,
                            const ParamDesc& p, void* rho_out, hipStream_t s) {
    const Brick br = brick_shape(g.nz);
    const int64_t blocks = int64_t((g.nx + br.bx - 1) / br.bx) * ((g.ny + br.by - 1) / br.by) *
                           ((g.nz + br.bz - 1) / br.bz);
    hipLaunchKernelGGL(sdf_build_kernel<T>, dim3(unsigned(blocks)), dim3(kSdfBlock), 0, s, q, n, w, ns, g, p,
                       static_cast<cplx<T>*>(rho_out));
    return hipGetLastError();
}

template hipError_t launch_sdf_build<float>(const double*, const double*, const double*, int64_t, const GridDesc&,
                                            const ParamDesc&, void*, hipStream_t);
template hipError_t launch_sdf_build<double>(const double*, const double*, const double*, int64_t, const GridDesc&,
                                             const ParamDesc&, void*, hipStream_t);

}  // namespace sdf
