// Skeletal density function on a grid (eq. 10A, 11, 12a, 13, 15, 16c, 17t).
//
// One thread per grid node; a block covers a compact 8 x 8 x 4 brick of
// nodes (16 x 16 in the plane) so that positions relative to the brick's
// corner are small.  Boundary samples stream through LDS in tiles of 256
// that every thread reads by broadcast.
//
// The samples are first put in Morton order (a stable radix sort of their
// quantised positions), so a tile of 256 consecutive samples covers a
// compact patch of the boundary, and every tile gets an FP64 bounding box.
// A brick then visits only the tiles that can matter to it:
//   pass 1: tiles whose box lies within U of the brick, where U is the least,
//           over all tiles, of the largest brick-to-tile-box distance (every
//           node of the brick has a sample within U);
//   pass 2: tiles whose box lies within (1 + eps) max xi_abs of the brick.
// Both bounds are conservative, so the nodes see exactly the samples they
// would see in a scan of all samples.
//
// Pass 1 finds the nearest sample (lowest original index on exact ties),
// its membership sign and the distance floor test.  These are discrete
// decisions, taken in FP64 from FP64 sample positions in both precisions,
// so the classification of every node is the one an FP64 evaluation makes.
//
// Pass 2 sums the kernel over the samples inside the eps-approximate contact
// ball, in the context's precision T, on brick-relative coordinates, in
// Morton order.  A sample whose squared distance lies within 1e-4 (relative)
// of the ball's squared radius is re-tested in FP64.
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

// A zero the compiler cannot see through: LDS addresses offset by it stay in
// a vector register across a loop, so the broadcast reads of the sample
// tiles use immediate offsets from it instead of re-copying a scalar base
// into a vector register for every read.
__device__ __forceinline__ int opaque_zero() {
    int z = 0;
    asm volatile("" : "+v"(z));
    return z;
}

// Samples in Morton order with per-tile bounding boxes.
struct SampleTiles {
    const double* qs;   // positions, n x 3
    const double* wn;   // w_j n_j, n x 3
    const int* js;      // original index of each sample
    const double* box;  // per tile of kSdfTile samples: lo x, y, z, hi x, y, z
    int64_t ntile;
};

__device__ __forceinline__ double box_dmin2(const double bl[3], const double bh[3], const double* __restrict__ t) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double d = fmax(0.0, fmax(t[a] - bh[a], bl[a] - t[3 + a]));
        s += d * d;
    }
    return s;
}
__device__ __forceinline__ double box_dmax2(const double bl[3], const double bh[3], const double* __restrict__ t) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double d = fmax(fabs(t[3 + a] - bl[a]), fabs(bh[a] - t[a]));
        s += d * d;
    }
    return s;
}

template <bool MAX>
__device__ __forceinline__ double block_reduce(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off);
        v = MAX ? fmax(v, o) : fmin(v, o);
    }
    __syncthreads();  // red is free
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    v = red[0];
#pragma unroll
    for (int wv = 1; wv < kSdfBlock / 64; ++wv) v = MAX ? fmax(v, red[wv]) : fmin(v, red[wv]);
    return v;
}

// Pass 1 (FP64) for the node (px, py, pz) of the brick [bl, bh]: squared
// distance to the nearest sample and its original index (lowest on exact
// ties), visiting only the tiles within U of the brick.  Block-wide: every
// thread of the block calls it.
__device__ __forceinline__ void nearest_pass(const SampleTiles& st, int64_t ns, const double bl[3], const double bh[3],
                                             double px, double py, double pz, v4<double>* sq, int* sidx, int* tflag,
                                             double* red, double& best, int& jbest, int64_t* visited = nullptr) {
    double u2 = INFINITY;
    for (int64_t t = threadIdx.x; t < st.ntile; t += kSdfBlock) u2 = fmin(u2, box_dmax2(bl, bh, st.box + 6 * t));
    u2 = block_reduce<false>(u2, red) * (1.0 + 1e-9);
    best = INFINITY;
    jbest = 0;
    for (int64_t c0 = 0; c0 < st.ntile; c0 += kSdfBlock) {
        const int64_t tc = c0 + threadIdx.x;
        __syncthreads();  // the previous chunk is done with tflag, sq and sidx
        tflag[threadIdx.x] = tc < st.ntile && box_dmin2(bl, bh, st.box + 6 * tc) <= u2;
        __syncthreads();
        const int nchunk = int(st.ntile - c0 < kSdfBlock ? st.ntile - c0 : kSdfBlock);
        for (int kk = 0; kk < nchunk; ++kk) {
            if (!tflag[kk]) continue;  // uniform across the block
            const int64_t t0 = (c0 + kk) * kSdfTile;
            const int cnt = int(ns - t0 < kSdfTile ? ns - t0 : kSdfTile);
            if (visited) *visited += cnt;
            __syncthreads();
            for (int a = threadIdx.x; a < cnt; a += kSdfBlock) {
                const int64_t s = t0 + a;
                sq[a] = v4<double>{st.qs[3 * s], st.qs[3 * s + 1], st.qs[3 * s + 2], 0.0};
                sidx[a] = st.js[s];
            }
            __syncthreads();
            const int z0 = opaque_zero();
            const v4<double>* sqb = sq + z0;
            const int* sib = sidx + z0;
#pragma unroll 4
            for (int a = 0; a < cnt; ++a) {
                const v4<double> s = sqb[a];
                const double dx = px - s.x, dy = py - s.y, dz = pz - s.z;
                const double d2 = dx * dx + dy * dy + dz * dz;
                const int jj = sib[a];
                if (d2 < best || (d2 == best && jj < jbest)) {
                    best = d2;
                    jbest = jj;
                }
            }
        }
    }
}

// PHI: the kernel of eq. 13 (kPhi* in launch.hpp): skeletal (eq. 15),
// inverse-square (eq. 15 with the medial Gaussian at its peak: the pair
// term without the exponential), or the double skin layer of eq. 3a, which
// needs only the signed distance of pass 1.
// STATS (measurement builds only): the block adds to stats[0..2] the
// node-sample pairs of pass 1 (valid nodes x samples of the visited tiles),
// of pass 2 (live nodes x samples of the visited tiles) and the pass-2 pairs
// inside the contact ball.
template <typename T, int PHI, bool STATS = false>
__global__ __launch_bounds__(kSdfBlock) void sdf_build_kernel(const double* __restrict__ q,
                                                              const double* __restrict__ nrm, SampleTiles st,
                                                              int64_t ns, GridDesc g, ParamDesc prm,
                                                              cplx<T>* __restrict__ out,
                                                              unsigned long long* __restrict__ stats = nullptr) {
    __shared__ v4<double> sq[2 * kSdfTile];  // pass 1: (qx, qy, qz, -); pass 2: reused as two T tiles
    __shared__ int sidx[kSdfTile];           // pass 1: original index; pass 2: Morton index
    __shared__ int tflag[kSdfBlock];         // tiles of the current chunk that the brick visits
    __shared__ double red[kSdfBlock / 64];
    v4<T>* sq2 = reinterpret_cast<v4<T>*>(sq);             // (qx, qy, qz, -) relative to the brick
    v4<T>* sn2 = reinterpret_cast<v4<T>*>(sq) + kSdfTile;  // w (nx, ny, nz), -

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
    // box of the brick's nodes inside the grid
    const double bl[3] = {cx, cy, cz};
    const double bh[3] = {cx + g.h * (min(br.bx, g.nx - i0) - 1), cy + g.h * (min(br.by, g.ny - j0) - 1),
                          cz + g.h * (min(br.bz, g.nz - k0) - 1)};

    // ---- pass 1 (FP64): nearest sample, lowest original index on exact ties
    double best;
    int jbest;
    int64_t vis1 = 0, vis2 = 0, inball = 0;
    nearest_pass(st, ns, bl, bh, px, py, pz, sq, sidx, tflag, red, best, jbest, STATS ? &vis1 : nullptr);
    const int64_t jb = jbest;
    const double dot = (px - q[3 * jb]) * nrm[3 * jb] + (py - q[3 * jb + 1]) * nrm[3 * jb + 1] +
                       (pz - q[3 * jb + 2]) * nrm[3 * jb + 2];
    const int pmc = dot > 0.0 ? 1 : (dot < 0.0 ? -1 : 0);
    const double xi_abs64 = sqrt(best);
    if constexpr (PHI == kPhiDsl) {
        // eq. 3a: lambda1 gb(xi / R - 1) + i lambda2 gb(xi / R + 1), FP64, defined
        // on the boundary too (no floor); gb truncates at |x| > eps
        if (valid) {
            const double xi = pmc * xi_abs64;
            const double x1 = xi / prm.radius - 1.0, x2 = xi / prm.radius + 1.0;
            const double c = 1.0 / (2.5066282746310002 * prm.sigma);
            const double h = -0.5 / (prm.sigma * prm.sigma);
            const double re = fabs(x1) <= prm.eps ? prm.lambda1 * c * exp(h * x1 * x1) : 0.0;
            const double im = fabs(x2) <= prm.eps ? prm.lambda2 * c * exp(h * x2 * x2) : 0.0;
            out[(int64_t(k) * g.ny + j) * g.nx + i] = mk(T(re), T(im));
        }
        return;
    }
    const bool live = valid && pmc != 0 && xi_abs64 >= prm.xi_floor;

    // ---- pass 2 (T): truncated kernel sum over the contact ball
    const double r2max64 = (1.0 + prm.eps) * (1.0 + prm.eps) * best;
    const double r2brick = block_reduce<true>(live ? r2max64 : -1.0, red) * (1.0 + 1e-9);
    const T r2lo = T(r2max64 * (1.0 - 1e-4)), r2hi = T(r2max64 * (1.0 + 1e-4));
    const T inv_xi = T(1.0 / xi_abs64);
    // exp(-(r - 1)^2 / (2 sigma^2)) = 2^(-u^2) with u = (r - 1) gs,
    // gs = sqrt(log2(e) / 2) / sigma, and u = eta (gs / xi) - gs
    const double gs64 = std::sqrt(0.5 * 1.4426950408889634) / prm.sigma;
    const T gs = T(gs64), inv_xi_gs = T(gs64 / xi_abs64);
    const T im_sign = pmc > 0 ? T(-2) : T(2);  // P = (1 - r^2) -+ 2 i r, applied once per node
    const T prx = T(rx), pry = T(ry), prz = T(rz);
    T acc_re = T(0), acc_im = T(0);
    if (r2brick >= 0.0) {  // uniform: some node of the brick is live
        for (int64_t c0 = 0; c0 < st.ntile; c0 += kSdfBlock) {
            const int64_t tc = c0 + threadIdx.x;
            __syncthreads();
            tflag[threadIdx.x] = tc < st.ntile && box_dmin2(bl, bh, st.box + 6 * tc) <= r2brick;
            __syncthreads();
            const int nchunk = int(st.ntile - c0 < kSdfBlock ? st.ntile - c0 : kSdfBlock);
            for (int kk = 0; kk < nchunk; ++kk) {
                if (!tflag[kk]) continue;  // uniform across the block
                const int64_t t0 = (c0 + kk) * kSdfTile;
                const int cnt = int(ns - t0 < kSdfTile ? ns - t0 : kSdfTile);
                if (STATS && live) vis2 += cnt;
                __syncthreads();
                for (int a = threadIdx.x; a < cnt; a += kSdfBlock) {
                    const int64_t s = t0 + a;
                    sq2[a] = v4<T>{T(st.qs[3 * s] - cx), T(st.qs[3 * s + 1] - cy), T(st.qs[3 * s + 2] - cz), T(0)};
                    sn2[a] = v4<T>{T(st.wn[3 * s]), T(st.wn[3 * s + 1]), T(st.wn[3 * s + 2]), T(0)};
                    sidx[a] = int(s);
                }
                __syncthreads();
                if (live) {
                    const int z0 = opaque_zero();
                    const v4<T>* sqb = sq2 + z0;
                    const v4<T>* snb = sn2 + z0;
#pragma unroll 4
                    for (int a = 0; a < cnt; ++a) {
                        const v4<T> s = sqb[a];
                        const T dx = prx - s.x, dy = pry - s.y, dz = prz - s.z;
                        const T d2 = dx * dx + dy * dy + dz * dz;
                        bool in = d2 <= r2lo;
                        if (!in && d2 <= r2hi) {  // near the sphere: decide in FP64
                            const int64_t sj = sidx[a];
                            const double ex = px - st.qs[3 * sj], ey = py - st.qs[3 * sj + 1],
                                         ez = pz - st.qs[3 * sj + 2];
                            in = ex * ex + ey * ey + ez * ez <= r2max64;
                        }
                        if (in) {
                            if (STATS) ++inball;
                            const v4<T> nv = snb[a];
                            const T inv_eta = fast_rsqrt(d2);
                            const T eta = d2 * inv_eta;
                            const T r = eta * inv_xi;
                            const T wcos = (dx * nv.x + dy * nv.y + dz * nv.z) * inv_eta;
                            T G = T(1);  // inverse-square: the medial Gaussian at its peak
                            if constexpr (PHI == kPhiSkeletal) {
                                const T u = eta * inv_xi_gs - gs;
                                G = dev_exp2(-u * u);
                            }
                            const T rr = r * r;
                            const T den = T(1) + rr;
                            const T coef = wcos * G * dev_rcp(den * den);
                            acc_re += coef * (T(1) - rr);
                            acc_im += coef * r;
                        }
                    }
                }
            }
        }
    }
    if constexpr (STATS) {
        // every thread walked the block's tiles: its pass-1 pairs are vis1
        // when its node is valid, its pass-2 pairs vis2 when live
        unsigned long long c[3] = {valid ? (unsigned long long)vis1 : 0ull, (unsigned long long)vis2,
                                   (unsigned long long)inball};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            for (int off = 32; off > 0; off >>= 1) c[a] += __shfl_xor(c[a], off);
            if ((threadIdx.x & 63) == 0) atomicAdd(stats + a, c[a]);
        }
    }
    if (valid) {
        cplx<T> res = mk(T(0), T(0));
        if (live) {
            const double lam = pmc > 0 ? prm.lambda1 : -prm.lambda2;
            const T scale = T(lam / (2.0 * 3.14159265358979323846 * prm.sigma * best));
            res = mk(acc_re * scale, acc_im * (im_sign * scale));
        }
        out[(int64_t(k) * g.ny + j) * g.nx + i] = res;
    }
}

// ---- radial-basis affinity (eq. 2, continuum form): Gaussian shells of
// radius R around the +R (skin) and -R (core) offsets of the boundary.
// The offset points come as samples whose "w n" slot holds their complex
// weight (lambda1 w, 0) or (0, lambda2 w); a node sums
//   c_j g_sigma(|p - s_j| / R - 1)  over |(|p - s_j| / R - 1)| <= eps,
// i.e. over the shell R max(0, 1 - eps) <= |p - s_j| <= R (1 + eps), whose
// edges are decided in FP64 (squared radii within 1e-4 are re-tested).
template <typename T>
__global__ __launch_bounds__(kSdfBlock) void sdf_radial_kernel(SampleTiles st, int64_t ns, GridDesc g,
                                                               ParamDesc prm, cplx<T>* __restrict__ out) {
    __shared__ v4<double> sq[2 * kSdfTile];
    __shared__ int sidx[kSdfTile];
    __shared__ int tflag[kSdfBlock];
    v4<T>* sq2 = reinterpret_cast<v4<T>*>(sq);             // (sx, sy, sz, -) relative to the brick
    v4<T>* sn2 = reinterpret_cast<v4<T>*>(sq) + kSdfTile;  // (c.re, c.im, -, -)

    const Brick br = brick_shape(g.nz);
    const int nbx = (g.nx + br.bx - 1) / br.bx, nby = (g.ny + br.by - 1) / br.by;
    const int blk = blockIdx.x;
    const int i0 = (blk % nbx) * br.bx, j0 = ((blk / nbx) % nby) * br.by, k0 = (blk / (nbx * nby)) * br.bz;
    const int li = threadIdx.x % br.bx, lj = (threadIdx.x / br.bx) % br.by, lk = threadIdx.x / (br.bx * br.by);
    const int i = i0 + li, j = j0 + lj, k = k0 + lk;
    const bool valid = i < g.nx && j < g.ny && k < g.nz;
    const double cx = g.ox + g.h * i0, cy = g.oy + g.h * j0, cz = g.oz + g.h * k0;
    const double rx = g.h * li, ry = g.h * lj, rz = g.h * lk;
    const double px = cx + rx, py = cy + ry, pz = cz + rz;
    const double bl[3] = {cx, cy, cz};
    const double bh[3] = {cx + g.h * (min(br.bx, g.nx - i0) - 1), cy + g.h * (min(br.by, g.ny - j0) - 1),
                          cz + g.h * (min(br.bz, g.nz - k0) - 1)};

    const double rhi = prm.radius * (1.0 + prm.eps);
    const double rlo = prm.eps < 1.0 ? prm.radius * (1.0 - prm.eps) : 0.0;
    const double hi2 = rhi * rhi, lo2 = rlo * rlo;
    const T hi2a = T(hi2 * (1.0 - 1e-4)), hi2b = T(hi2 * (1.0 + 1e-4));
    const T lo2a = T(lo2 * (1.0 - 1e-4)), lo2b = T(lo2 * (1.0 + 1e-4));
    // g_sigma(eta / R - 1) = 2^(-u^2) / (sqrt(2 pi) sigma), u = (eta / R - 1) gs
    const double gs64 = std::sqrt(0.5 * 1.4426950408889634) / prm.sigma;
    const T gs = T(gs64), inv_r_gs = T(gs64 / prm.radius);
    const T prx = T(rx), pry = T(ry), prz = T(rz);
    T acc_re = T(0), acc_im = T(0);
    for (int64_t c0 = 0; c0 < st.ntile; c0 += kSdfBlock) {
        const int64_t tc = c0 + threadIdx.x;
        __syncthreads();
        tflag[threadIdx.x] = tc < st.ntile && box_dmin2(bl, bh, st.box + 6 * tc) <= hi2 * (1.0 + 1e-9) &&
                             !(box_dmax2(bl, bh, st.box + 6 * tc) < lo2 * (1.0 - 1e-9));
        __syncthreads();
        const int nchunk = int(st.ntile - c0 < kSdfBlock ? st.ntile - c0 : kSdfBlock);
        for (int kk = 0; kk < nchunk; ++kk) {
            if (!tflag[kk]) continue;  // uniform across the block
            const int64_t t0 = (c0 + kk) * kSdfTile;
            const int cnt = int(ns - t0 < kSdfTile ? ns - t0 : kSdfTile);
            __syncthreads();
            for (int a = threadIdx.x; a < cnt; a += kSdfBlock) {
                const int64_t s = t0 + a;
                sq2[a] = v4<T>{T(st.qs[3 * s] - cx), T(st.qs[3 * s + 1] - cy), T(st.qs[3 * s + 2] - cz), T(0)};
                sn2[a] = v4<T>{T(st.wn[3 * s]), T(st.wn[3 * s + 1]), T(0), T(0)};
                sidx[a] = int(s);
            }
            __syncthreads();
            if (valid) {
#pragma unroll 4
                for (int a = 0; a < cnt; ++a) {
                    const v4<T> sp = sq2[a];
                    const T dx = prx - sp.x, dy = pry - sp.y, dz = prz - sp.z;
                    const T d2 = dx * dx + dy * dy + dz * dz;
                    bool in = d2 <= hi2a && d2 >= lo2b;
                    if (!in && d2 <= hi2b && d2 >= lo2a) {  // near a shell edge: decide in FP64
                        const int64_t sj = sidx[a];
                        const double ex = px - st.qs[3 * sj], ey = py - st.qs[3 * sj + 1], ez = pz - st.qs[3 * sj + 2];
                        const double e2 = ex * ex + ey * ey + ez * ez;
                        in = e2 <= hi2 && e2 >= lo2;
                    }
                    if (in) {
                        const v4<T> cw = sn2[a];
                        const T u = sqrt(d2) * inv_r_gs - gs;
                        const T G = dev_exp2(-u * u);
                        acc_re += cw.x * G;
                        acc_im += cw.y * G;
                    }
                }
            }
        }
    }
    if (valid) {
        const T c = T(1.0 / (2.5066282746310002 * prm.sigma));
        out[(int64_t(k) * g.ny + j) * g.nx + i] = mk(acc_re * c, acc_im * c);
    }
}

// skin (+R n_j, weight (lambda1 w_j, 0)) and core (-R n_j, (0, lambda2 w_j))
// offset points of the samples, FP64, as a sample set of 2n points
__global__ void offset_points_kernel(const double* __restrict__ q, const double* __restrict__ nrm,
                                     const double* __restrict__ w, int64_t n, double R, double l1, double l2,
                                     double* __restrict__ q2, double* __restrict__ c2, double* __restrict__ w2) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= n) return;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        q2[3 * j + a] = q[3 * j + a] + R * nrm[3 * j + a];
        q2[3 * (n + j) + a] = q[3 * j + a] - R * nrm[3 * j + a];
    }
    c2[3 * j] = l1;
    c2[3 * j + 1] = 0.0;
    c2[3 * j + 2] = 0.0;
    c2[3 * (n + j)] = 0.0;
    c2[3 * (n + j) + 1] = l2;
    c2[3 * (n + j) + 2] = 0.0;
    w2[j] = w[j];
    w2[n + j] = w[j];
}

// ---- adjoint with respect to the boundary samples
// L = Re sum_p g(p) rho(p).  With the nearest sample, membership and contact
// ball of every node held (FP64 throughout; the cotangent g comes in the
// context's precision), at a live node with nearest sample q* at xi:
//   d rho / d w_j = A c_j K(r_j),   d rho / d n_j = A w_j K(r_j) u_j,
//   d rho / d q_j = A w_j [-K(r_j) (n_j - c_j u_j) / eta_j - c_j K'(r_j) u_j / xi],
//   d rho / d xi  = -(2 rho + A sum_j w_j c_j K'(r_j) r_j) / xi,   d xi / d q* = -u*,
// with A = lambda / (2 pi sigma xi^2), K = G P / (1 + r^2)^2 as in the sum and
//   K' = K (-(r - 1) / sigma^2 - 4 r / (1 + r^2)) + G (-2 r + i s) / (1 + r^2)^2.
__device__ __forceinline__ void kernel_and_slope(double r, double sig2inv, double s, double& kre, double& kim,
                                                 double& dre, double& dim) {
    const double x = r - 1.0;
    const double G = exp(-0.5 * x * x * sig2inv);
    const double iden = 1.0 / (1.0 + r * r);
    const double gi = G * iden * iden;
    kre = gi * (1.0 - r * r);
    kim = gi * (s * r);
    const double f = -x * sig2inv - 4.0 * r * iden;
    dre = kre * f - 2.0 * r * gi;
    dim = kim * f + s * gi;
}

// A block per brick.  Pass 1 as in the build; a node pass over the contact
// ball gives rho and the xi term, added to the nearest sample's position
// gradient; a sample pass puts the brick's live nodes in LDS, and each
// thread owns one sample of a visited tile and sums its gradient over those
// nodes.  Sums across bricks go through FP64 atomics (their order varies, so
// the last bits of the gradients may vary between runs).
template <typename T>
__global__ __launch_bounds__(kSdfBlock) void sdf_adjoint_kernel(const double* __restrict__ q,
                                                                const double* __restrict__ nrm,
                                                                const double* __restrict__ w, SampleTiles st,
                                                                int64_t ns, GridDesc g, ParamDesc prm,
                                                                const cplx<T>* __restrict__ cot,
                                                                double* __restrict__ gq, double* __restrict__ gn,
                                                                double* __restrict__ gw) {
    __shared__ v4<double> sq[2 * kSdfTile];
    __shared__ int sidx[kSdfTile];
    __shared__ int tflag[kSdfBlock];
    __shared__ double red[kSdfBlock / 64];
    __shared__ v4<double> nodep[kSdfBlock];  // (px, py, pz, 1 / xi)
    __shared__ v4<double> nodeg[kSdfBlock];  // (A g.re, A g.im, ball radius^2 or -1, s)
    static_assert(kSdfTile == kSdfBlock, "one sample per thread in the sample pass");

    const Brick br = brick_shape(g.nz);
    const int nbx = (g.nx + br.bx - 1) / br.bx, nby = (g.ny + br.by - 1) / br.by;
    const int blk = blockIdx.x;
    const int i0 = (blk % nbx) * br.bx, j0 = ((blk / nbx) % nby) * br.by, k0 = (blk / (nbx * nby)) * br.bz;
    const int li = threadIdx.x % br.bx, lj = (threadIdx.x / br.bx) % br.by, lk = threadIdx.x / (br.bx * br.by);
    const int i = i0 + li, j = j0 + lj, k = k0 + lk;
    const bool valid = i < g.nx && j < g.ny && k < g.nz;
    const double cx = g.ox + g.h * i0, cy = g.oy + g.h * j0, cz = g.oz + g.h * k0;
    const double px = cx + g.h * li, py = cy + g.h * lj, pz = cz + g.h * lk;
    const double bl[3] = {cx, cy, cz};
    const double bh[3] = {cx + g.h * (min(br.bx, g.nx - i0) - 1), cy + g.h * (min(br.by, g.ny - j0) - 1),
                          cz + g.h * (min(br.bz, g.nz - k0) - 1)};

    double best;
    int jbest;
    nearest_pass(st, ns, bl, bh, px, py, pz, sq, sidx, tflag, red, best, jbest);
    const int64_t jb = jbest;
    const double ex = px - q[3 * jb], ey = py - q[3 * jb + 1], ez = pz - q[3 * jb + 2];
    const double dot = ex * nrm[3 * jb] + ey * nrm[3 * jb + 1] + ez * nrm[3 * jb + 2];
    const int pmc = dot > 0.0 ? 1 : (dot < 0.0 ? -1 : 0);
    const double xi = sqrt(best);
    const cplx<T> gt = valid ? cot[(int64_t(k) * g.ny + j) * g.nx + i] : mk(T(0), T(0));
    const double g_re = double(gt.re), g_im = double(gt.im);
    const bool act = valid && pmc != 0 && xi >= prm.xi_floor && (g_re != 0.0 || g_im != 0.0);
    const double r2max = (1.0 + prm.eps) * (1.0 + prm.eps) * best;
    const double lam = pmc > 0 ? prm.lambda1 : -prm.lambda2;
    const double sgn = pmc > 0 ? -2.0 : 2.0;
    const double A = lam / (2.0 * 3.14159265358979323846 * prm.sigma * best);
    const double inv_xi = 1.0 / xi;
    const double sig2inv = 1.0 / (prm.sigma * prm.sigma);
    const double r2brick = block_reduce<true>(act ? r2max : -1.0, red) * (1.0 + 1e-9);
    if (r2brick < 0.0) return;  // uniform: no node of the brick contributes

    // ---- node pass: rho / A and sum_j w_j c_j K'(r_j) r_j over the ball
    double rr = 0.0, ri = 0.0, sr = 0.0, si = 0.0;
    for (int64_t c0 = 0; c0 < st.ntile; c0 += kSdfBlock) {
        const int64_t tc = c0 + threadIdx.x;
        __syncthreads();
        tflag[threadIdx.x] = tc < st.ntile && box_dmin2(bl, bh, st.box + 6 * tc) <= r2brick;
        __syncthreads();
        const int nchunk = int(st.ntile - c0 < kSdfBlock ? st.ntile - c0 : kSdfBlock);
        for (int kk = 0; kk < nchunk; ++kk) {
            if (!tflag[kk]) continue;  // uniform across the block
            const int64_t t0 = (c0 + kk) * kSdfTile;
            const int cnt = int(ns - t0 < kSdfTile ? ns - t0 : kSdfTile);
            __syncthreads();
            for (int a = threadIdx.x; a < cnt; a += kSdfBlock) {
                const int64_t s = t0 + a;
                sq[a] = v4<double>{st.qs[3 * s], st.qs[3 * s + 1], st.qs[3 * s + 2], 0.0};
                sq[kSdfTile + a] = v4<double>{st.wn[3 * s], st.wn[3 * s + 1], st.wn[3 * s + 2], 0.0};
            }
            __syncthreads();
            if (act) {
                for (int a = 0; a < cnt; ++a) {
                    const v4<double> sp = sq[a];
                    const double dx = px - sp.x, dy = py - sp.y, dz = pz - sp.z;
                    const double d2 = dx * dx + dy * dy + dz * dz;
                    if (d2 <= r2max) {
                        const v4<double> wv = sq[kSdfTile + a];
                        const double ie = rsqrt(d2);
                        const double eta = d2 * ie;
                        const double wc = (dx * wv.x + dy * wv.y + dz * wv.z) * ie;  // w_j c_j
                        const double r = eta * inv_xi;
                        double kre, kim, dre, dim;
                        kernel_and_slope(r, sig2inv, sgn, kre, kim, dre, dim);
                        rr += wc * kre;
                        ri += wc * kim;
                        sr += wc * dre * r;
                        si += wc * dim * r;
                    }
                }
            }
        }
    }
    if (act) {
        // d rho / d xi = -(2 A rr + A sr) / xi (complex), then Re(g ...) along -u*
        const double dre = -A * (2.0 * rr + sr) * inv_xi, dim = -A * (2.0 * ri + si) * inv_xi;
        const double coef = (g_re * dre - g_im * dim) * inv_xi;
        atomicAdd(gq + 3 * jb, -coef * ex);
        atomicAdd(gq + 3 * jb + 1, -coef * ey);
        atomicAdd(gq + 3 * jb + 2, -coef * ez);
    }

    // ---- sample pass: the brick's live nodes in LDS, one sample per thread.
    // Every brick is resident at once, so each starts its walk over the tiles
    // at its own offset: bricks then add to different samples' gradients at a
    // time instead of contending for the same addresses.
    __syncthreads();
    nodep[threadIdx.x] = v4<double>{px, py, pz, inv_xi};
    nodeg[threadIdx.x] = v4<double>{A * g_re, A * g_im, act ? r2max : -1.0, sgn};
    const int64_t nchunks = (st.ntile + kSdfBlock - 1) / kSdfBlock;
    for (int64_t ci = 0; ci < nchunks; ++ci) {
        const int64_t c0 = ((ci + blk) % nchunks) * kSdfBlock;
        const int64_t tc = c0 + threadIdx.x;
        __syncthreads();
        tflag[threadIdx.x] = tc < st.ntile && box_dmin2(bl, bh, st.box + 6 * tc) <= r2brick;
        __syncthreads();
        const int nchunk = int(st.ntile - c0 < kSdfBlock ? st.ntile - c0 : kSdfBlock);
        for (int k1 = 0; k1 < nchunk; ++k1) {
            const int kk = (k1 + blk) % nchunk;
            if (!tflag[kk]) continue;  // uniform across the block
            const int64_t t0 = (c0 + kk) * kSdfTile;
            const int cnt = int(ns - t0 < kSdfTile ? ns - t0 : kSdfTile);
            if (int(threadIdx.x) >= cnt) continue;
            const int64_t sj = st.js[t0 + threadIdx.x];
            const double qx = q[3 * sj], qy = q[3 * sj + 1], qz = q[3 * sj + 2];
            const double nx = nrm[3 * sj], ny = nrm[3 * sj + 1], nz = nrm[3 * sj + 2];
            const double wj = w[sj];
            double aq0 = 0.0, aq1 = 0.0, aq2 = 0.0, an0 = 0.0, an1 = 0.0, an2 = 0.0, aw = 0.0;
            bool any = false;
            for (int nd = 0; nd < kSdfBlock; ++nd) {
                const v4<double> ng = nodeg[nd];
                if (ng.z < 0.0) continue;  // the same node for every thread: uniform
                const v4<double> np = nodep[nd];
                const double dx = np.x - qx, dy = np.y - qy, dz = np.z - qz;
                const double d2 = dx * dx + dy * dy + dz * dz;
                if (d2 > ng.z) continue;
                any = true;
                const double ie = rsqrt(d2);
                const double ux = dx * ie, uy = dy * ie, uz = dz * ie;
                const double c = ux * nx + uy * ny + uz * nz;
                const double r = d2 * ie * np.w;
                double kre, kim, dre, dim;
                kernel_and_slope(r, sig2inv, ng.w, kre, kim, dre, dim);
                const double gk = ng.x * kre - ng.y * kim;    // Re(A g K)
                const double gkp = ng.x * dre - ng.y * dim;   // Re(A g K')
                aw += c * gk;
                const double wg = wj * gk;
                an0 += wg * ux;
                an1 += wg * uy;
                an2 += wg * uz;
                const double t1 = -wg * ie, t2 = -wj * c * gkp * np.w;
                aq0 += t1 * (nx - c * ux) + t2 * ux;
                aq1 += t1 * (ny - c * uy) + t2 * uy;
                aq2 += t1 * (nz - c * uz) + t2 * uz;
            }
            if (any) {
                atomicAdd(gq + 3 * sj, aq0);
                atomicAdd(gq + 3 * sj + 1, aq1);
                atomicAdd(gq + 3 * sj + 2, aq2);
                atomicAdd(gn + 3 * sj, an0);
                atomicAdd(gn + 3 * sj + 1, an1);
                atomicAdd(gn + 3 * sj + 2, an2);
                atomicAdd(gw + sj, aw);
            }
        }
    }
}

// ---- Morton order and tile boxes
__device__ __forceinline__ unsigned spread10(unsigned x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

// 10 bits per axis over the grid's box widened by 4 h (outside samples clamp)
__global__ void morton_key_kernel(const double* __restrict__ q, int64_t n, double ox, double oy, double oz,
                                  double inv_cell, unsigned* __restrict__ key, int* __restrict__ val) {
    const int64_t jx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (jx >= n) return;
    const double o[3] = {ox, oy, oz};
    unsigned c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double f = (q[3 * jx + a] - o[a]) * inv_cell;
        c[a] = !(f > 0.0) ? 0u : (f >= 1023.0 ? 1023u : unsigned(f));
    }
    key[jx] = spread10(c[0]) | (spread10(c[1]) << 1) | (spread10(c[2]) << 2);
    val[jx] = int(jx);
}

__global__ void sample_gather_kernel(const double* __restrict__ q, const double* __restrict__ nrm,
                                     const double* __restrict__ w, const int* __restrict__ order, int64_t n,
                                     double* __restrict__ qs, double* __restrict__ wn) {
    const int64_t ix = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (ix >= n) return;
    const int64_t s = order[ix];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        qs[3 * ix + a] = q[3 * s + a];
        wn[3 * ix + a] = w[s] * nrm[3 * s + a];
    }
}

__global__ void tile_box_kernel(const double* __restrict__ qs, int64_t n, int64_t ntile, double* __restrict__ box) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= ntile) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int64_t e = (t + 1) * kSdfTile < n ? (t + 1) * kSdfTile : n;
    for (int64_t s = t * kSdfTile; s < e; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fmin(lo[a], qs[3 * s + a]);
            hi[a] = fmax(hi[a], qs[3 * s + a]);
        }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        box[6 * t + a] = lo[a];
        box[6 * t + 3 + a] = hi[a];
    }
}

// workspace carve-up (256-byte aligned pieces)
struct SdfWs {
    size_t keys_in, vals_in, keys_out, vals_out, qs, wn, box, temp, temp_bytes, total;
};
inline size_t al256(size_t b) { return (b + 255) / 256 * 256; }
inline SdfWs sdf_ws_layout(int64_t n) {
    SdfWs L{};
    const size_t temp_bytes = sort_temp_bytes(n);
    const int64_t ntile = (n + kSdfTile - 1) / kSdfTile;
    size_t off = 0;
    L.keys_in = off;
    off += al256(size_t(n) * 4);
    L.vals_in = off;
    off += al256(size_t(n) * 4);
    L.keys_out = off;
    off += al256(size_t(n) * 4);
    L.vals_out = off;
    off += al256(size_t(n) * 4);
    L.qs = off;
    off += al256(size_t(n) * 24);
    L.wn = off;
    off += al256(size_t(n) * 24);
    L.box = off;
    off += al256(size_t(ntile) * 48);
    L.temp = off;
    L.temp_bytes = temp_bytes;
    off += al256(temp_bytes);
    L.total = off;
    return L;
}

// Morton order, sorted copies and tile boxes in the workspace
hipError_t prepare_tiles(const double* q, const double* n, const double* w, int64_t ns, const GridDesc& g, void* ws,
                         hipStream_t s, SampleTiles* st) {
    const SdfWs L = sdf_ws_layout(ns);
    char* base = static_cast<char*>(ws);
    auto* keys_in = reinterpret_cast<unsigned*>(base + L.keys_in);
    auto* vals_in = reinterpret_cast<int*>(base + L.vals_in);
    auto* keys_out = reinterpret_cast<unsigned*>(base + L.keys_out);
    auto* vals_out = reinterpret_cast<int*>(base + L.vals_out);
    auto* qs = reinterpret_cast<double*>(base + L.qs);
    auto* wn = reinterpret_cast<double*>(base + L.wn);
    auto* box = reinterpret_cast<double*>(base + L.box);
    const int64_t ntile = (ns + kSdfTile - 1) / kSdfTile;
    const unsigned gb = unsigned((ns + 255) / 256);
    const double ext = g.h * (std::max(g.nx, std::max(g.ny, g.nz)) + 8);
    hipLaunchKernelGGL(morton_key_kernel, dim3(gb), dim3(256), 0, s, q, ns, g.ox - 4 * g.h, g.oy - 4 * g.h,
                       g.oz - 4 * g.h, 1024.0 / ext, keys_in, vals_in);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned* keys_sorted = nullptr;
    int* order = nullptr;
    e = launch_sort_pairs(keys_in, vals_in, keys_out, vals_out, ns, 30, base + L.temp, s, &keys_sorted, &order);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sample_gather_kernel, dim3(gb), dim3(256), 0, s, q, n, w, order, ns, qs, wn);
    hipLaunchKernelGGL(tile_box_kernel, dim3(unsigned((ntile + 63) / 64)), dim3(64), 0, s, qs, ns, ntile, box);
    *st = SampleTiles{qs, wn, order, box, ntile};
    return hipGetLastError();
}

int64_t brick_count(const GridDesc& g) {
    const Brick br = brick_shape(g.nz);
    return int64_t((g.nx + br.bx - 1) / br.bx) * ((g.ny + br.by - 1) / br.by) * ((g.nz + br.bz - 1) / br.bz);
}

}  // namespace

size_t sdf_build_workspace_bytes(int64_t ns, int phi) {
    // the radial kernel tiles the 2 n offset points, held (positions, weight
    // slots, weights) ahead of the tile layout
    if (phi == kPhiRadial) return al256(size_t(ns) * 2 * 7 * sizeof(double)) + sdf_ws_layout(2 * ns).total;
    return sdf_ws_layout(ns).total;
}

template <typename T>
hipError_t launch_sdf_build(const double* q, const double* n, const double* w, int64_t ns, const GridDesc& g,
                            const ParamDesc& p, int phi, void* rho_out, void* ws, hipStream_t s,
                            unsigned long long* stats) {
    SampleTiles st{};
    const dim3 grid(unsigned(brick_count(g))), block(kSdfBlock);
    auto* out = static_cast<cplx<T>*>(rho_out);
    if (phi == kPhiRadial) {
        double* q2 = static_cast<double*>(ws);
        double* c2 = q2 + 6 * ns;
        double* w2 = c2 + 6 * ns;
        hipLaunchKernelGGL(offset_points_kernel, dim3(unsigned((ns + 255) / 256)), dim3(256), 0, s, q, n, w, ns,
                           p.radius, p.lambda1, p.lambda2, q2, c2, w2);
        void* ws2 = static_cast<char*>(ws) + al256(size_t(ns) * 2 * 7 * sizeof(double));
        hipError_t e = prepare_tiles(q2, c2, w2, 2 * ns, g, ws2, s, &st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(sdf_radial_kernel<T>, grid, block, 0, s, st, 2 * ns, g, p, out);
        return hipGetLastError();
    }
    hipError_t e = prepare_tiles(q, n, w, ns, g, ws, s, &st);
    if (e != hipSuccess) return e;
    if (stats) {
        hipLaunchKernelGGL((sdf_build_kernel<T, kPhiSkeletal, true>), grid, block, 0, s, q, n, st, ns, g, p, out,
                           stats);
        return hipGetLastError();
    }
    if (phi == kPhiDsl)
        hipLaunchKernelGGL((sdf_build_kernel<T, kPhiDsl>), grid, block, 0, s, q, n, st, ns, g, p, out);
    else if (phi == kPhiInverseSquare)
        hipLaunchKernelGGL((sdf_build_kernel<T, kPhiInverseSquare>), grid, block, 0, s, q, n, st, ns, g, p, out);
    else
        hipLaunchKernelGGL((sdf_build_kernel<T, kPhiSkeletal>), grid, block, 0, s, q, n, st, ns, g, p, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sdf_adjoint(const double* q, const double* n, const double* w, int64_t ns, const GridDesc& g,
                              const ParamDesc& p, const void* cot, double* grad_q, double* grad_n, double* grad_w,
                              void* ws, hipStream_t s) {
    // zeroed by a kernel, not hipMemsetAsync, so the call can be captured in a graph
    hipError_t e = launch_zero_f64(grad_q, 3 * ns, s);
    if (e == hipSuccess) e = launch_zero_f64(grad_n, 3 * ns, s);
    if (e == hipSuccess) e = launch_zero_f64(grad_w, ns, s);
    if (e != hipSuccess) return e;
    SampleTiles st{};
    e = prepare_tiles(q, n, w, ns, g, ws, s, &st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sdf_adjoint_kernel<T>, dim3(unsigned(brick_count(g))), dim3(kSdfBlock), 0, s, q, n, w, st,
                       ns, g, p, static_cast<const cplx<T>*>(cot), grad_q, grad_n, grad_w);
    return hipGetLastError();
}

template hipError_t launch_sdf_adjoint<float>(const double*, const double*, const double*, int64_t, const GridDesc&,
                                              const ParamDesc&, const void*, double*, double*, double*, void*,
                                              hipStream_t);
template hipError_t launch_sdf_adjoint<double>(const double*, const double*, const double*, int64_t,
                                               const GridDesc&, const ParamDesc&, const void*, double*, double*,
                                               double*, void*, hipStream_t);
template hipError_t launch_sdf_build<float>(const double*, const double*, const double*, int64_t, const GridDesc&,
                                            const ParamDesc&, int, void*, void*, hipStream_t, unsigned long long*);
template hipError_t launch_sdf_build<double>(const double*, const double*, const double*, int64_t, const GridDesc&,
                                             const ParamDesc&, int, void*, void*, hipStream_t, unsigned long long*);

}  // namespace sdf
