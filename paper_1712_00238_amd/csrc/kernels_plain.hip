// Plain multi-pass correlation path, one template for FP32 and FP64:
//   quaternions -> rotation matrices (FP64), c_k = w_k rho_M(x_k),
//   spread with global atomics, per-axis LDS FFT passes, pointwise product
//   with the fixed spectrum, inverse passes, Re + peak reduction.
// Every step is a separate launch over whole grids; this is the
// straightforward baseline the fused FP32 kernels are measured against.
#include "common.hpp"
#include "fft.hpp"
#include "fft256.hpp"
#include "launch.hpp"

namespace sdf {

namespace {

// ------------------------------------------------------------------ rotations
template <typename T>
__global__ void quat_to_rot_kernel(const double* __restrict__ quats, int64_t n, double* __restrict__ r64,
                                   T* __restrict__ rT) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double w = quats[4 * i], x = quats[4 * i + 1], y = quats[4 * i + 2], z = quats[4 * i + 3];
    double inv = 1.0 / sqrt(w * w + x * x + y * y + z * z);
    w *= inv;
    x *= inv;
    y *= inv;
    z *= inv;
    double r[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z),     2 * (x * z + w * y),
                   2 * (x * y + w * z),     1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                   2 * (x * z - w * y),     2 * (y * z + w * x),     1 - 2 * (x * x + y * y)};
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        if (r64) r64[9 * i + a] = r[a];
        if (rT) rT[9 * i + a] = T(r[a]);
    }
}

template <typename T>
__global__ void coef_kernel(const cplx<T>* __restrict__ rho, const T* __restrict__ w, int64_t n,
                            cplx<T>* __restrict__ c) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) c[i] = rho[i] * w[i];
}

template <typename T>
__global__ void zero_kernel(cplx<T>* __restrict__ p, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) p[i] = mk(T(0), T(0));
}

// ------------------------------------------------------------------ spread
// One thread per body sample: y = sign * R (k - n_m/2), 4^3 (planar: 4^2)
// B-spline stencil, periodic, accumulated with global atomics.
template <typename T>
__global__ void spread_atomic_kernel(const cplx<T>* __restrict__ c, int n_m, int planar, const T* __restrict__ R,
                                     T sign, int N, cplx<T>* __restrict__ out) {
    const int64_t K = planar ? int64_t(n_m) * n_m : int64_t(n_m) * n_m * n_m;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const cplx<T> ck = c[k];
    if (ck.re == T(0) && ck.im == T(0)) return;
    const int rot = blockIdx.y;
    const T* r = R + 9 * rot;
    const T half = T(0.5) * T(n_m);
    const T bx = T(int(k % n_m)) - half;
    const T by = T(int((k / n_m) % n_m)) - half;
    const T bz = planar ? T(0) : T(int(k / (int64_t(n_m) * n_m))) - half;
    const T yx = sign * (r[0] * bx + r[1] * by + r[2] * bz);
    const T yy = sign * (r[3] * bx + r[4] * by + r[5] * bz);
    const T yz = sign * (r[6] * bx + r[7] * by + r[8] * bz);
    const T fx0 = dev_floor(yx), fy0 = dev_floor(yy);
    T wx[4], wy[4], wz[4];
    bspline3_weights(yx - fx0, wx);
    bspline3_weights(yy - fy0, wy);
    const int ix = int(fx0) - 1, iy = int(fy0) - 1;
    const int64_t gsz = planar ? int64_t(N) * N : int64_t(N) * N * N;
    cplx<T>* g = out + rot * gsz;
    if (planar) {
        for (int b = 0; b < 4; ++b) {
            const int yy_i = wrap(iy + b, N);
            for (int a = 0; a < 4; ++a) {
                const int xx_i = wrap(ix + a, N);
                const T wt = wx[a] * wy[b];
                cplx<T>* p = g + int64_t(yy_i) * N + xx_i;
                atomicAdd(&p->re, ck.re * wt);
                atomicAdd(&p->im, ck.im * wt);
            }
        }
        return;
    }
    const T fz0 = dev_floor(yz);
    bspline3_weights(yz - fz0, wz);
    const int iz = int(fz0) - 1;
    for (int cz = 0; cz < 4; ++cz) {
        const int zz_i = wrap(iz + cz, N);
        for (int b = 0; b < 4; ++b) {
            const int yy_i = wrap(iy + b, N);
            const T wyz = wy[b] * wz[cz];
            for (int a = 0; a < 4; ++a) {
                const int xx_i = wrap(ix + a, N);
                const T wt = wx[a] * wyz;
                cplx<T>* p = g + (int64_t(zz_i) * N + yy_i) * N + xx_i;
                atomicAdd(&p->re, ck.re * wt);
                atomicAdd(&p->im, ck.im * wt);
            }
        }
    }
}

// ------------------------------------------------------------------ direct reference
// Boundary samples of the moving part turned about its body-box centre c:
// q' = c + R (q - c), n' = R n (FP64, R row-major).
__global__ void rotate_samples_kernel(const double* __restrict__ q, const double* __restrict__ nrm, int64_t ns,
                                      const double* __restrict__ R, double cx, double cy, double cz,
                                      double* __restrict__ qo, double* __restrict__ no) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= ns) return;
    const double d[3] = {q[3 * j] - cx, q[3 * j + 1] - cy, q[3 * j + 2] - cz};
    const double c[3] = {cx, cy, cz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        qo[3 * j + a] = c[a] + R[3 * a] * d[0] + R[3 * a + 1] * d[1] + R[3 * a + 2] * d[2];
        no[3 * j + a] = R[3 * a] * nrm[3 * j] + R[3 * a + 1] * nrm[3 * j + 1] + R[3 * a + 2] * nrm[3 * j + 2];
    }
}

// Body-box values placed on the fixed grid without a window, reflected as
// the spread with sign -1 places them: node k (body position k - n_m / 2,
// n_m even) goes to u = -(k - n_m / 2) mod N.  Distinct nodes land on
// distinct grid nodes (n_m <= N), so plain stores suffice.
template <typename T>
__global__ void place_direct_kernel(const cplx<T>* __restrict__ rho, int n_m, int planar, T w_node, int N,
                                    cplx<T>* __restrict__ out) {
    const int64_t K = planar ? int64_t(n_m) * n_m : int64_t(n_m) * n_m * n_m;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const int h = n_m / 2;
    const int kx = int(k % n_m), ky = int((k / n_m) % n_m), kz = planar ? h : int(k / (int64_t(n_m) * n_m));
    const int ux = wrap(h - kx, N), uy = wrap(h - ky, N), uz = planar ? 0 : wrap(h - kz, N);
    out[(int64_t(uz) * N + uy) * N + ux] = rho[k] * w_node;
}

// ------------------------------------------------------------------ FFT passes

constexpr int kFftBlock = 256;

// Rows (x axis, contiguous): a block transforms conc = 256 / (N/8) rows.
template <typename T, int N, int S>
__global__ __launch_bounds__(kFftBlock) void fft_rows_kernel(cplx<T>* __restrict__ data, int64_t nrows, T scale) {
    constexpr int TPL = FFTShape<N>::TPL;
    constexpr int CONC = kFftBlock / TPL;
    __shared__ cplx<T> buf[CONC * N];
    __shared__ cplx<T> tw[N];
    fill_twiddles<T, N>(tw);
    const int64_t row0 = int64_t(blockIdx.x) * CONC;
    const int nr = int(nrows - row0 < CONC ? nrows - row0 : CONC);
    cplx<T>* src = data + row0 * N;
    for (int i = threadIdx.x; i < nr * N; i += kFftBlock) buf[i] = src[i];
    __syncthreads();
    lds_fft_lines<T, N, S, false>(buf, 1, N, nr, tw);
    for (int i = threadIdx.x; i < nr * N; i += kFftBlock) src[i] = buf[i] * scale;
}

// Columns per block for the strided passes: the largest power of two that
// fits the block's lines and divides N.
template <int N>
constexpr int cols_width() {
    int w = 1;
    while (w * 2 <= kFftBlock / FFTShape<N>::TPL && N % (w * 2) == 0) w *= 2;
    return w;
}

// Strided axis (y: es = N, z: es = N^2): a block takes W consecutive x
// columns of one (other-axis) plane and transforms them along the axis.
template <typename T, int N, int S>
__global__ __launch_bounds__(kFftBlock) void fft_cols_kernel(cplx<T>* __restrict__ data, int64_t es, int64_t os,
                                                             int64_t gsz, T scale) {
    constexpr int W = cols_width<N>();
    __shared__ cplx<T> buf[N * W];
    __shared__ cplx<T> tw[N];
    fill_twiddles<T, N>(tw);
    const int x0 = blockIdx.x * W;
    const int o = blockIdx.y;
    cplx<T>* base = data + int64_t(blockIdx.z) * gsz + int64_t(o) * os + x0;
    for (int i = threadIdx.x; i < N * W; i += kFftBlock) {
        const int e = i / W, xl = i % W;
        buf[i] = base[e * es + xl];
    }
    __syncthreads();
    lds_fft_lines<T, N, S, true>(buf, W, 1, W, tw);
    for (int i = threadIdx.x; i < N * W; i += kFftBlock) {
        const int e = i / W, xl = i % W;
        base[e * es + xl] = buf[i] * scale;
    }
}

template <typename T, int N>
hipError_t fft3_impl(void* data, bool planar, int batch, int dir, double scale, hipStream_t s) {
    constexpr int TPL = FFTShape<N>::TPL;
    constexpr int CONC = kFftBlock / TPL;
    constexpr int W = cols_width<N>();
    cplx<T>* d = static_cast<cplx<T>*>(data);
    const int nz = planar ? 1 : N;
    const int64_t gsz = int64_t(N) * N * nz;
    const int64_t nrows = int64_t(N) * nz * batch;
    const T one = T(1), sc = T(scale);
    // x
    {
        dim3 grid(unsigned((nrows + CONC - 1) / CONC));
        if (dir < 0)
            hipLaunchKernelGGL((fft_rows_kernel<T, N, -1>), grid, dim3(kFftBlock), 0, s, d, nrows, one);
        else
            hipLaunchKernelGGL((fft_rows_kernel<T, N, 1>), grid, dim3(kFftBlock), 0, s, d, nrows, one);
    }
    // y: columns of each z plane
    {
        dim3 grid(N / W, nz, batch);
        const T scy = planar ? sc : one;
        if (dir < 0)
            hipLaunchKernelGGL((fft_cols_kernel<T, N, -1>), grid, dim3(kFftBlock), 0, s, d, int64_t(N),
                               int64_t(N) * N, gsz, scy);
        else
            hipLaunchKernelGGL((fft_cols_kernel<T, N, 1>), grid, dim3(kFftBlock), 0, s, d, int64_t(N),
                               int64_t(N) * N, gsz, scy);
    }
    // z: columns of each y row
    if (!planar) {
        dim3 grid(N / W, N, batch);
        if (dir < 0)
            hipLaunchKernelGGL((fft_cols_kernel<T, N, -1>), grid, dim3(kFftBlock), 0, s, d, int64_t(N) * N,
                               int64_t(N), gsz, sc);
        else
            hipLaunchKernelGGL((fft_cols_kernel<T, N, 1>), grid, dim3(kFftBlock), 0, s, d, int64_t(N) * N,
                               int64_t(N), gsz, sc);
    }
    return hipGetLastError();
}

template <typename T>
__global__ void mul_spec_kernel(cplx<T>* __restrict__ data, const cplx<T>* __restrict__ spec, int64_t count,
                                int batch) {
    const int64_t total = count * batch;
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (; i < total; i += stride) data[i] = data[i] * spec[i % count];
}

// ------------------------------------------------------------------ peak
constexpr int kPeakBlock = 256;

template <typename T>
__device__ __forceinline__ bool better(T v, int i, T bv, int bi) {
    return v > bv || (v == bv && i < bi);
}

template <typename T>
__device__ __forceinline__ void block_argmax(T& v, int& idx) {
    __shared__ T sv[kPeakBlock];
    __shared__ int si[kPeakBlock];
    sv[threadIdx.x] = v;
    si[threadIdx.x] = idx;
    __syncthreads();
    for (int off = int(blockDim.x) / 2; off > 0; off >>= 1) {
        if (int(threadIdx.x) < off) {
            T ov = sv[threadIdx.x + off];
            int oi = si[threadIdx.x + off];
            if (better(ov, oi, sv[threadIdx.x], si[threadIdx.x])) {
                sv[threadIdx.x] = ov;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    v = sv[0];
    idx = si[0];
    __syncthreads();
}

template <typename T, bool CPLX>
__device__ __forceinline__ T vol_at(const void* vol, int64_t i) {
    if (CPLX) return static_cast<const cplx<T>*>(vol)[i].re;
    return static_cast<const T*>(vol)[i];
}

template <typename T, bool CPLX>
__global__ __launch_bounds__(kPeakBlock) void peak_partial_kernel(const void* __restrict__ vol, int64_t nvox,
                                                                  int nparts, T* __restrict__ pval,
                                                                  int* __restrict__ pidx) {
    const int part = blockIdx.x, b = blockIdx.y;
    const int64_t chunk = (nvox + nparts - 1) / nparts;
    const int64_t lo = part * chunk;
    const int64_t hi = lo + chunk < nvox ? lo + chunk : nvox;
    const int64_t off = int64_t(b) * nvox;
    T bv = T(-INFINITY);
    int bi = 0x7fffffff;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kPeakBlock) {
        T v = vol_at<T, CPLX>(vol, off + i);
        if (better(v, int(i), bv, bi)) {
            bv = v;
            bi = int(i);
        }
    }
    block_argmax(bv, bi);
    if (threadIdx.x == 0) {
        pval[int64_t(b) * nparts + part] = bv;
        pidx[int64_t(b) * nparts + part] = bi;
    }
}

template <typename T, bool CPLX>
__global__ __launch_bounds__(kPeakBlock) void peak_final_kernel(const void* __restrict__ vol, int N, int planar,
                                                                int nparts, const T* __restrict__ pval,
                                                                const int* __restrict__ pidx, T* __restrict__ score,
                                                                int32_t* __restrict__ tout, T* __restrict__ nbhd,
                                                                double* __restrict__ refined) {
    const int b = blockIdx.x;
    const int nz = planar ? 1 : N;
    const int64_t nvox = int64_t(N) * N * nz;
    T bv = T(-INFINITY);
    int bi = 0x7fffffff;
    for (int i = threadIdx.x; i < nparts; i += kPeakBlock) {
        T v = pval[int64_t(b) * nparts + i];
        int id = pidx[int64_t(b) * nparts + i];
        if (better(v, id, bv, bi)) {
            bv = v;
            bi = id;
        }
    }
    block_argmax(bv, bi);
    __shared__ T nb[27];
    const int tx = bi % N, ty = (bi / N) % N, tz = bi / (N * N);
    if (threadIdx.x < 27) {
        const int dz = threadIdx.x / 9 - 1, dy = (threadIdx.x / 3) % 3 - 1, dx = threadIdx.x % 3 - 1;
        const int zz = wrap(tz + dz, nz), yy = wrap(ty + dy, N), xx = wrap(tx + dx, N);
        nb[threadIdx.x] = vol_at<T, CPLX>(vol, int64_t(b) * nvox + (int64_t(zz) * N + yy) * N + xx);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        score[b] = bv;
        tout[3 * b] = tx;
        tout[3 * b + 1] = ty;
        tout[3 * b + 2] = tz;
        if (nbhd)
            for (int a = 0; a < 27; ++a) nbhd[27 * int64_t(b) + a] = nb[a];
        if (refined) {
            // per-axis parabola through (f-, f0, f+), FP64
            const double f0 = double(nb[13]);
            const double fm[3] = {double(nb[12]), double(nb[10]), double(nb[4])};
            const double fp[3] = {double(nb[14]), double(nb[16]), double(nb[22])};
            const int ti[3] = {tx, ty, tz};
            for (int a = 0; a < 3; ++a) {
                const double den = fm[a] - 2.0 * f0 + fp[a];
                double d = 0.0;
                if (den < 0.0) {
                    d = (fm[a] - fp[a]) / (2.0 * den);
                    d = d < -0.5 ? -0.5 : (d > 0.5 ? 0.5 : d);
                }
                refined[3 * b + a] = double(ti[a]) + d;
            }
        }
    }
}

template <typename T>
__global__ void real_part_kernel(const cplx<T>* __restrict__ v, T* __restrict__ out, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (; i < n; i += stride) out[i] = v[i].re;
}

inline unsigned grid_for(int64_t n, int block, int cap = 65535 * 4) {
    int64_t g = (n + block - 1) / block;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return unsigned(g);
}

}  // namespace

template <typename T>
hipError_t launch_quat_to_rot(const double* quats, int64_t n, double* r64, T* rT, hipStream_t s) {
    hipLaunchKernelGGL(quat_to_rot_kernel<T>, dim3(grid_for(n, 64)), dim3(64), 0, s, quats, n, r64, rT);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coef(const void* rho_m, const T* w_m, int64_t count, void* c_out, hipStream_t s) {
    hipLaunchKernelGGL(coef_kernel<T>, dim3(unsigned((count + 255) / 256)), dim3(256), 0, s,
                       static_cast<const cplx<T>*>(rho_m), w_m, count, static_cast<cplx<T>*>(c_out));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_zero(void* buf, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(zero_kernel<T>, dim3(grid_for(count, 256, 16384)), dim3(256), 0, s,
                       static_cast<cplx<T>*>(buf), count);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_spread_atomic(const void* c, int n_m, bool planar, const T* R, int n_rot, T sign, int N, void* out,
                                hipStream_t s) {
    const int64_t K = planar ? int64_t(n_m) * n_m : int64_t(n_m) * n_m * n_m;
    dim3 grid(unsigned((K + 255) / 256), unsigned(n_rot));
    hipLaunchKernelGGL(spread_atomic_kernel<T>, grid, dim3(256), 0, s, static_cast<const cplx<T>*>(c), n_m,
                       planar ? 1 : 0, R, sign, N, static_cast<cplx<T>*>(out));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fft3(void* data, int N, bool planar, int batch, int dir, double scale, hipStream_t s) {
    switch (N) {
        case 8: return fft3_impl<T, 8>(data, planar, batch, dir, scale, s);
        case 16: return fft3_impl<T, 16>(data, planar, batch, dir, scale, s);
        case 32: return fft3_impl<T, 32>(data, planar, batch, dir, scale, s);
        case 64: return fft3_impl<T, 64>(data, planar, batch, dir, scale, s);
        case 96: return fft3_impl<T, 96>(data, planar, batch, dir, scale, s);
        case 128: return fft3_impl<T, 128>(data, planar, batch, dir, scale, s);
        case 256: return fft3_impl<T, 256>(data, planar, batch, dir, scale, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_mul_spec(void* data, const void* spec, int64_t count, int batch, hipStream_t s) {
    hipLaunchKernelGGL(mul_spec_kernel<T>, dim3(grid_for(count * batch, 256, 16384)), dim3(256), 0, s,
                       static_cast<cplx<T>*>(data), static_cast<const cplx<T>*>(spec), count, batch);
    return hipGetLastError();
}

template <typename T>
int peak_parts(int N, bool planar) {
    const int64_t nvox = int64_t(N) * N * (planar ? 1 : N);
    int64_t p = (nvox + 4095) / 4096;
    if (p > 512) p = 512;
    if (p < 1) p = 1;
    return int(p);
}

template <typename T>
hipError_t launch_peak(const void* vol, bool vol_is_complex, int N, bool planar, int batch, T* part_val,
                       int* part_idx, int nparts, T* score, int32_t* t, T* nbhd, double* refined, hipStream_t s) {
    const int64_t nvox = int64_t(N) * N * (planar ? 1 : N);
    const dim3 g1{unsigned(nparts), unsigned(batch), 1u};
    if (vol_is_complex) {
        hipLaunchKernelGGL((peak_partial_kernel<T, true>), g1, dim3(kPeakBlock), 0, s, vol, nvox, nparts, part_val,
                           part_idx);
        hipLaunchKernelGGL((peak_final_kernel<T, true>), dim3(unsigned(batch)), dim3(kPeakBlock), 0, s, vol, N,
                           planar ? 1 : 0, nparts, part_val, part_idx, score, t, nbhd, refined);
    } else {
        hipLaunchKernelGGL((peak_partial_kernel<T, false>), g1, dim3(kPeakBlock), 0, s, vol, nvox, nparts,
                           part_val, part_idx);
        hipLaunchKernelGGL((peak_final_kernel<T, false>), dim3(unsigned(batch)), dim3(kPeakBlock), 0, s, vol, N,
                           planar ? 1 : 0, nparts, part_val, part_idx, score, t, nbhd, refined);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_real_part(const void* vol, T* out, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(real_part_kernel<T>, dim3(grid_for(count, 256, 16384)), dim3(256), 0, s,
                       static_cast<const cplx<T>*>(vol), out, count);
    return hipGetLastError();
}

hipError_t launch_rotate_samples(const double* q, const double* nrm, int64_t ns, const double* R, const double c[3],
                                 double* qo, double* no, hipStream_t s) {
    hipLaunchKernelGGL(rotate_samples_kernel, dim3(unsigned((ns + 255) / 256)), dim3(256), 0, s, q, nrm, ns, R, c[0],
                       c[1], c[2], qo, no);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_place_direct(const void* rho, int n_m, bool planar, T w_node, int N, void* out, hipStream_t s) {
    const int64_t K = planar ? int64_t(n_m) * n_m : int64_t(n_m) * n_m * n_m;
    hipLaunchKernelGGL(place_direct_kernel<T>, dim3(unsigned((K + 255) / 256)), dim3(256), 0, s,
                       static_cast<const cplx<T>*>(rho), n_m, planar ? 1 : 0, w_node, N, static_cast<cplx<T>*>(out));
    return hipGetLastError();
}

#define SDF_INST(T)                                                                                              \
    template hipError_t launch_quat_to_rot<T>(const double*, int64_t, double*, T*, hipStream_t);                \
    template hipError_t launch_coef<T>(const void*, const T*, int64_t, void*, hipStream_t);                      \
    template hipError_t launch_zero<T>(void*, int64_t, hipStream_t);                                             \
    template hipError_t launch_place_direct<T>(const void*, int, bool, T, int, void*, hipStream_t);               \
    template hipError_t launch_spread_atomic<T>(const void*, int, bool, const T*, int, T, int, void*,           \
                                                hipStream_t);                                                    \
    template hipError_t launch_fft3<T>(void*, int, bool, int, int, double, hipStream_t);                         \
    template hipError_t launch_mul_spec<T>(void*, const void*, int64_t, int, hipStream_t);                       \
    template int peak_parts<T>(int, bool);                                                                      \
    template hipError_t launch_peak<T>(const void*, bool, int, bool, int, T*, int*, int, T*, int32_t*, T*,      \
                                       double*, hipStream_t);                                                    \
    template hipError_t launch_real_part<T>(const void*, T*, int64_t, hipStream_t);

SDF_INST(float)
SDF_INST(double)

}  // namespace sdf
