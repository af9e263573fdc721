// Pose value and adjoint for gradient-based refinement of placements.
//
//   f(t, q) = Re sum_k c_k Phi(R x_k / h + t),  Phi(y) = sum_p rho_F(p) B3(p - y),
//   df/dt   = Re sum_k c_k grad Phi(y_k),
//   df/dR   = G = sum_k Re(c_k grad Phi(y_k)) (x_k / h)^T,  df/dq = G : dR/dq,
//   df/dw_k = sum_b s_b Re(rho_M(x_k) Phi_b(y_k)).
//
// Block (sample tile, pose tile): each thread owns a few body samples and
// walks the poses of the tile, gathering the 4^3 stencil of rho_F around
// each moved sample (the stencil weights are recomputed here, never stored).
// Per pose the 13 sums (f, df/dt, G) are accumulated in FP64 and reduced
// per block into partials; a second kernel reduces the partials per pose and
// applies the quaternion chain rule in FP64.  Per-sample weight gradients
// stay in registers across the pose tile and are written once per tile.
#include "common.hpp"
#include "launch.hpp"

namespace sdf {

namespace {

constexpr int kGBlock = 256;
constexpr int kSPT = 4;                        // samples per thread
constexpr int kSamplesPerBlock = kGBlock * kSPT;
constexpr int kPosesPerBlock = 16;
constexpr int kNAcc = 13;  // f, dt[3], G[9]

__device__ __forceinline__ void quat_rot(const double* q, double r[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    const double inv = 1.0 / sqrt(w * w + x * x + y * y + z * z);
    w *= inv;
    x *= inv;
    y *= inv;
    z *= inv;
    r[0] = 1 - 2 * (y * y + z * z);
    r[1] = 2 * (x * y - w * z);
    r[2] = 2 * (x * z + w * y);
    r[3] = 2 * (x * y + w * z);
    r[4] = 1 - 2 * (x * x + z * z);
    r[5] = 2 * (y * z - w * x);
    r[6] = 2 * (x * z - w * y);
    r[7] = 2 * (y * z + w * x);
    r[8] = 1 - 2 * (x * x + y * y);
}

__device__ __forceinline__ double warp_sum(double v) {
    for (int off = warpSize / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

template <typename T, bool GRAD>
__global__ __launch_bounds__(kGBlock) void grad_tile_kernel(const cplx<T>* __restrict__ rho_f, int N, int planar,
                                                            const cplx<T>* __restrict__ rho_m,
                                                            const T* __restrict__ w_m, int n_m,
                                                            const double* __restrict__ poses, int64_t B,
                                                            const double* __restrict__ gscale,
                                                            double* __restrict__ part, int nsb,
                                                            T* __restrict__ wpart, int want_w) {
    const int sb = blockIdx.x, pb = blockIdx.y;
    const int64_t K = planar ? int64_t(n_m) * n_m : int64_t(n_m) * n_m * n_m;
    const int nz = planar ? 1 : N;
    const T half = T(0.5) * T(n_m);

    // this thread's samples
    int64_t ks[kSPT];
    T xb[kSPT][3];
    cplx<T> ck[kSPT], rm[kSPT];
    T gw[kSPT];
#pragma unroll
    for (int s = 0; s < kSPT; ++s) {
        const int64_t k = int64_t(sb) * kSamplesPerBlock + s * kGBlock + threadIdx.x;
        ks[s] = k;
        const int64_t kk = k < K ? k : 0;
        xb[s][0] = T(int(kk % n_m)) - half;
        xb[s][1] = T(int((kk / n_m) % n_m)) - half;
        xb[s][2] = planar ? T(0) : T(int(kk / (int64_t(n_m) * n_m))) - half;
        rm[s] = k < K ? rho_m[kk] : mk(T(0), T(0));
        ck[s] = rm[s] * (k < K ? w_m[kk] : T(0));
        gw[s] = T(0);
    }

    __shared__ double red[kGBlock / 64][kNAcc];
    const int lane = threadIdx.x % warpSize, wid = threadIdx.x / warpSize;

    const int64_t b0 = int64_t(pb) * kPosesPerBlock;
    for (int pi = 0; pi < kPosesPerBlock; ++pi) {
        const int64_t b = b0 + pi;
        if (b >= B) break;  // uniform across the block
        const double* pose = poses + 7 * b;
        double r64[9];
        quat_rot(pose + 3, r64);
        T r[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) r[a] = T(r64[a]);
        // split t into an integer and a fractional part so that positions are
        // formed in the sample's local frame (keeps FP32 stencils accurate)
        double tint[3];
        T tfr[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            tint[a] = floor(pose[a]);
            tfr[a] = T(pose[a] - tint[a]);
        }
        const double sc = gscale ? gscale[b] : 1.0;
        double acc[kNAcc];
#pragma unroll
        for (int a = 0; a < kNAcc; ++a) acc[a] = 0.0;

#pragma unroll
        for (int s = 0; s < kSPT; ++s) {
            if (ks[s] >= K) continue;
            T y[3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
                y[a] = tfr[a] + r[3 * a] * xb[s][0] + r[3 * a + 1] * xb[s][1] + r[3 * a + 2] * xb[s][2];
            T fl[3], wgt[3][4], dw[3][4];
            int base[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                fl[a] = dev_floor(y[a]);
                base[a] = int(fl[a]) + int(tint[a]) - 1;
                bspline3_weights(y[a] - fl[a], wgt[a]);
                if (GRAD) bspline3_dweights(y[a] - fl[a], dw[a]);
            }
            cplx<T> phi = mk(T(0), T(0)), gx = phi, gy = phi, gz = phi;
            const int zc = planar ? 1 : 4;
            for (int cz = 0; cz < zc; ++cz) {
                const int iz = planar ? 0 : wrap(base[2] + cz, nz);
                const T wz = planar ? T(1) : wgt[2][cz];
                const T dz = planar ? T(0) : (GRAD ? dw[2][cz] : T(0));
#pragma unroll
                for (int cy = 0; cy < 4; ++cy) {
                    const int iy = wrap(base[1] + cy, N);
                    const cplx<T>* row = rho_f + (int64_t(iz) * N + iy) * N;
                    cplx<T> rx = mk(T(0), T(0)), rdx = rx;
#pragma unroll
                    for (int cx = 0; cx < 4; ++cx) {
                        const cplx<T> v = row[wrap(base[0] + cx, N)];
                        rx = rx + v * wgt[0][cx];
                        if (GRAD) rdx = rdx + v * dw[0][cx];
                    }
                    phi = phi + rx * (wgt[1][cy] * wz);
                    if (GRAD) {
                        gx = gx + rdx * (wgt[1][cy] * wz);
                        gy = gy + rx * (dw[1][cy] * wz);
                        gz = gz + rx * (wgt[1][cy] * dz);
                    }
                }
            }
            const cplx<T> v = ck[s] * phi;
            acc[0] += double(v.re);
            if (GRAD) {
                const double g0 = double((ck[s] * gx).re), g1 = double((ck[s] * gy).re),
                             g2 = double((ck[s] * gz).re);
                acc[1] += g0;
                acc[2] += g1;
                acc[3] += g2;
                const double x0 = double(xb[s][0]), x1 = double(xb[s][1]), x2 = double(xb[s][2]);
                acc[4] += g0 * x0;
                acc[5] += g0 * x1;
                acc[6] += g0 * x2;
                acc[7] += g1 * x0;
                acc[8] += g1 * x1;
                acc[9] += g1 * x2;
                acc[10] += g2 * x0;
                acc[11] += g2 * x1;
                acc[12] += g2 * x2;
                if (want_w) gw[s] += T(sc) * (rm[s] * phi).re;
            }
        }
        // block reduction of the per-pose sums (FP64)
        const int nacc = GRAD ? kNAcc : 1;
        for (int a = 0; a < nacc; ++a) {
            double v = warp_sum(acc[a]);
            if (lane == 0) red[wid][a] = v;
        }
        __syncthreads();
        if (threadIdx.x < nacc) {
            double v = 0.0;
            for (int wv = 0; wv < kGBlock / 64; ++wv) v += red[wv][threadIdx.x];
            part[(b * nsb + sb) * kNAcc + threadIdx.x] = v;
        }
        __syncthreads();
    }
    if (GRAD && want_w) {
#pragma unroll
        for (int s = 0; s < kSPT; ++s)
            if (ks[s] < K) wpart[int64_t(pb) * K + ks[s]] = gw[s];
    }
}

// Per pose: reduce the sample-tile partials, apply the chain rule through
// R(q / |q|) (FP64), write the score and the 7 pose derivatives.
template <typename T, bool GRAD>
__global__ void grad_finish_kernel(const double* __restrict__ part, int nsb, const double* __restrict__ poses,
                                   int64_t B, T* __restrict__ score, double* __restrict__ grad_pose) {
    const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double acc[kNAcc];
    for (int a = 0; a < kNAcc; ++a) acc[a] = 0.0;
    const int nacc = GRAD ? kNAcc : 1;
    for (int sb = 0; sb < nsb; ++sb)
        for (int a = 0; a < nacc; ++a) acc[a] += part[(b * nsb + sb) * kNAcc + a];
    score[b] = T(acc[0]);
    if (!GRAD || !grad_pose) return;
    const double* q = poses + 7 * b + 3;
    const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double w = q[0] / nq, x = q[1] / nq, y = q[2] / nq, z = q[3] / nq;
    // dR_ab / du_c, u = q / |q|, c = (w, x, y, z)
    const double d[9][4] = {{0, 0, -4 * y, -4 * z},          {-2 * z, 2 * y, 2 * x, -2 * w},
                            {2 * y, 2 * z, 2 * w, 2 * x},    {2 * z, 2 * y, 2 * x, 2 * w},
                            {0, -4 * x, 0, -4 * z},          {-2 * x, -2 * w, 2 * z, 2 * y},
                            {-2 * y, 2 * z, -2 * w, 2 * x},  {2 * x, 2 * w, 2 * z, 2 * y},
                            {0, -4 * x, -4 * y, 0}};
    double gu[4] = {0, 0, 0, 0};
    for (int ab = 0; ab < 9; ++ab)
        for (int c = 0; c < 4; ++c) gu[c] += acc[4 + ab] * d[ab][c];
    // d/dq = (I - u u^T) / |q| applied to d/du
    const double u[4] = {w, x, y, z};
    const double ug = u[0] * gu[0] + u[1] * gu[1] + u[2] * gu[2] + u[3] * gu[3];
    double* g = grad_pose + 7 * b;
    g[0] = acc[1];
    g[1] = acc[2];
    g[2] = acc[3];
    for (int c = 0; c < 4; ++c) g[3 + c] = (gu[c] - u[c] * ug) / nq;
}

template <typename T>
__global__ void wsum_kernel(const T* __restrict__ wpart, int npb, int64_t K, T* __restrict__ grad_w) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= K) return;
    T s = T(0);
    for (int p = 0; p < npb; ++p) s += wpart[int64_t(p) * K + k];
    grad_w[k] = s;
}

}  // namespace

template <typename T>
size_t grad_workspace_bytes(int64_t B, int n_m, bool planar, bool want_w) {
    const int64_t K = planar ? int64_t(n_m) * n_m : int64_t(n_m) * n_m * n_m;
    const int64_t nsb = (K + kSamplesPerBlock - 1) / kSamplesPerBlock;
    const int64_t npb = (B + kPosesPerBlock - 1) / kPosesPerBlock;
    size_t bytes = size_t(B * nsb * kNAcc) * sizeof(double);
    bytes = (bytes + 255) / 256 * 256;
    if (want_w) bytes += size_t(npb * K) * sizeof(T);
    return bytes + 256;
}

template <typename T>
hipError_t launch_score_grad(const void* rho_f, int N, bool planar, const void* rho_m, const T* w_m, int n_m,
                             const double* poses, int64_t B, T* score, double* grad_pose, T* grad_w,
                             const double* grad_scale, void* ws, hipStream_t s) {
    const int64_t K = planar ? int64_t(n_m) * n_m : int64_t(n_m) * n_m * n_m;
    const int nsb = int((K + kSamplesPerBlock - 1) / kSamplesPerBlock);
    const int npb = int((B + kPosesPerBlock - 1) / kPosesPerBlock);
    double* part = static_cast<double*>(ws);
    size_t off = size_t(B * nsb * kNAcc) * sizeof(double);
    off = (off + 255) / 256 * 256;
    T* wpart = reinterpret_cast<T*>(static_cast<char*>(ws) + off);
    const bool grad = grad_pose != nullptr || grad_w != nullptr;
    const dim3 grid{unsigned(nsb), unsigned(npb), 1u};
    const auto* rf = static_cast<const cplx<T>*>(rho_f);
    const auto* rm = static_cast<const cplx<T>*>(rho_m);
    if (grad)
        hipLaunchKernelGGL((grad_tile_kernel<T, true>), grid, dim3(kGBlock), 0, s, rf, N, planar ? 1 : 0, rm, w_m, n_m,
                           poses, B, grad_scale, part, nsb, wpart, grad_w ? 1 : 0);
    else
        hipLaunchKernelGGL((grad_tile_kernel<T, false>), grid, dim3(kGBlock), 0, s, rf, N, planar ? 1 : 0, rm, w_m,
                           n_m, poses, B, grad_scale, part, nsb, wpart, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 g2(unsigned((B + 127) / 128));
    if (grad)
        hipLaunchKernelGGL((grad_finish_kernel<T, true>), g2, dim3(128), 0, s, part, nsb, poses, B, score, grad_pose);
    else
        hipLaunchKernelGGL((grad_finish_kernel<T, false>), g2, dim3(128), 0, s, part, nsb, poses, B, score, nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (grad_w) {
        hipLaunchKernelGGL(wsum_kernel<T>, dim3(unsigned((K + 255) / 256)), dim3(256), 0, s, wpart, npb, K, grad_w);
        e = hipGetLastError();
    }
    return e;
}

template size_t grad_workspace_bytes<float>(int64_t, int, bool, bool);
template size_t grad_workspace_bytes<double>(int64_t, int, bool, bool);
template hipError_t launch_score_grad<float>(const void*, int, bool, const void*, const float*, int, const double*,
                                             int64_t, float*, double*, float*, const double*, void*, hipStream_t);
template hipError_t launch_score_grad<double>(const void*, int, bool, const void*, const double*, int, const double*,
                                              int64_t, double*, double*, double*, const double*, void*, hipStream_t);

}  // namespace sdf
