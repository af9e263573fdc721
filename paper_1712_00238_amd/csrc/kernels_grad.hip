// Pose value and adjoint for gradient-based refinement of placements.
//
//   f(t, q) = Re sum_k c_k Phi(R x_k / h + t),  Phi(y) = sum_p rho_F(p) B3(p - y),
//   df/dt   = Re sum_k c_k grad Phi(y_k)                      (g_k = Re c_k grad Phi(y_k)),
//   df/dq   from the torque tau = sum_k (R x_k / h) x g_k:    for a unit quaternion u the
//             rotated point moves by 2 vec(e_c u*) x (R x) + (radial part) along u_c,
//             so df/du_c = 2 vec(e_c u*) . tau on the tangent space of |u| = 1,
//   df/dw_k = sum_b s_b Re(rho_M(x_k) Phi_b(y_k)).
//
// Block (sample tile, pose tile): threads own body samples and walk the poses
// of the tile, gathering the 4^3 stencil of rho_F around each moved sample
// (the stencil weights are recomputed here, never stored).  Per pose the 7
// sums (f, df/dt, tau) are accumulated in FP64 and reduced per block into
// partials; a second kernel reduces the partials per pose and applies the
// quaternion chain rule in FP64.  Per-sample weight gradients stay in
// registers across the pose tile and are written once per tile.
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "launch.hpp"

namespace sdf {

namespace {

constexpr int kGBlock = 256;
constexpr int kSPT = 4;                        // samples per thread
constexpr int kSamplesPerBlock = kGBlock * kSPT;
constexpr int kPosesPerBlock = 16;
constexpr int kNAcc = 7;  // f, dt[3], tau[3]

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
                                                            T* __restrict__ wpart, int want_w, int pb0) {
    const int sb = blockIdx.x, pb = pb0 + int(blockIdx.y);
    const int64_t K = planar ? int64_t(n_m) * n_m : int64_t(n_m) * n_m * n_m;
    const int nz = planar ? 1 : N;
    const T half = T(0.5) * T(n_m);

    // this thread's samples
    int64_t ks[kSPT];
    T xb[kSPT][3];
    cplx<T> ck[kSPT], rm[kSPT];
    T gw[kSPT], gwi[kSPT];  // wmode 1: Re(rho_M Phi) sums; 2: Phi sums (re, im)
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
        gwi[s] = T(0);
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
                // rotated body position R x (without t) and torque (R x) x g
                double wv[3];
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    wv[a] = double(r[3 * a]) * double(xb[s][0]) + double(r[3 * a + 1]) * double(xb[s][1]) +
                            double(r[3 * a + 2]) * double(xb[s][2]);
                acc[4] += wv[1] * g2 - wv[2] * g1;
                acc[5] += wv[2] * g0 - wv[0] * g2;
                acc[6] += wv[0] * g1 - wv[1] * g0;
                if (want_w == 1) gw[s] += T(sc) * (rm[s] * phi).re;
                if (want_w == 2) {
                    gw[s] += T(sc) * phi.re;
                    gwi[s] += T(sc) * phi.im;
                }
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
            if (ks[s] < K) {
                if (want_w == 1) wpart[int64_t(pb) * K + ks[s]] = gw[s];
                else {
                    wpart[2 * (int64_t(pb) * K + ks[s])] = gw[s];
                    wpart[2 * (int64_t(pb) * K + ks[s]) + 1] = gwi[s];
                }
            }
    }
}

// Sum of v over each row of 16 lanes, left in every lane of the row (DPP
// quad permutations and row rotations; no LDS traffic).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row16_sum(double v) {
    v += dpp_f64<0xb1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4e>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x124>(v);  // row_ror 4
    v += dpp_f64<0x128>(v);  // row_ror 8
    return v;
}

// 3D FP32 variant with the fixed field staged in LDS.  Block (8 x 8 x 8
// sample tile, pose tile), one sample per thread.  Per pose the block loads
// into LDS the box of rho_F cells that the tile's 4^3 stencils can touch:
// the tile's corners bound its moved positions (widened by 1e-3 cell, far
// above the FP32 rounding of a moved position), so the stencil floors span at
// most ceil(7 |row of R|_1) + 1 <= 14 values and the box is at most 17 cells
// per axis.  The box has fixed pitches (18 cells per row, 312 per plane: of
// the pitches timed, the best over both uniformly spread and clustered
// rotations, whose stencil gathers meet different LDS bank conflicts), so the
// 64 stencil reads of a sample sit at constant offsets from one address.
// Staging gives each wave three box rows per load instruction (54 lanes, row
// and plane on the scalar unit) and issues all of a wave's loads before its
// LDS stores.
constexpr int kBoxTile = 8;
constexpr int kBoxBlock = kBoxTile * kBoxTile * kBoxTile;
constexpr int kBoxWaves = kBoxBlock / 64;
constexpr int kBoxMax = 17;
constexpr int kBoxRow = 18;
constexpr int kBoxPlane = 312;
constexpr int kBoxCells = kBoxPlane * kBoxMax;
constexpr int kBoxSlotRows = 3;                                            // rows per wave load
constexpr int kBoxSlots = kBoxMax * ((kBoxMax + kBoxSlotRows - 1) / kBoxSlotRows);
constexpr int kBoxStage = (kBoxSlots + kBoxWaves - 1) / kBoxWaves;         // loads per lane
constexpr int kBoxPoses = 16;
constexpr float kBoxMargin = 1e-3f;
static_assert(kBoxRow >= kBoxMax && kBoxPlane >= kBoxRow * kBoxMax, "box pitches");
static_assert(kBoxRow * kBoxSlotRows <= 64, "staging rows per wave");

// Per-pose constants of the box kernel, computed once per pose: R in FP32,
// t split into floor and fraction, and the offsets of the moved 8^3 tile's
// bounding box from its moved corner, sum_c min(0, 7 R_ac) and
// sum_c max(0, 7 R_ac).
struct BoxPose {
    float r[9];
    float tfr[3];
    int tint[3];
    float dmin[3];
    float dmax[3];
    float pad[3];
};
static_assert(sizeof(BoxPose) == 96, "BoxPose layout");

__global__ void box_pose_kernel(const double* __restrict__ poses, int64_t B, BoxPose* __restrict__ out) {
    const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double* pose = poses + 7 * b;
    double r64[9];
    quat_rot(pose + 3, r64);
    BoxPose P;
#pragma unroll
    for (int a = 0; a < 9; ++a) P.r[a] = float(r64[a]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double ti = floor(pose[a]);
        P.tint[a] = int(ti);
        P.tfr[a] = float(pose[a] - ti);
        float lo = 0.f, hi = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float e = float(kBoxTile - 1) * P.r[3 * a + c];
            lo += fminf(e, 0.f);
            hi += fmaxf(e, 0.f);
        }
        P.dmin[a] = lo;
        P.dmax[a] = hi;
        P.pad[a] = 0.f;
    }
    out[b] = P;
}

// REAL (pose gradients without weight gradients): only Re(c_k Phi) and the
// real parts of c_k times Phi's derivatives are needed, so the stencil
// contracts u = Re(c_k v) per cell, one real product chain instead of a
// complex one from the y sums on (16 fewer VALU instructions per plane).
template <bool GRAD, bool REAL = false>
__global__ __launch_bounds__(kBoxBlock, 2) void grad_box_kernel(const cplx<float>* __restrict__ rho_f, int N,
                                                                const cplx<float>* __restrict__ rho_m,
                                                                const float* __restrict__ w_m, int n_m,
                                                                const BoxPose* __restrict__ bpose, int64_t B,
                                                                const double* __restrict__ gscale,
                                                                double* __restrict__ part, int nsb,
                                                                float* __restrict__ wpart, int want_w, int pb0) {
    __shared__ cplx<float> box[kBoxCells];
    __shared__ double red[kBoxBlock / 16][kNAcc];
    const int sb = blockIdx.x, pb = pb0 + int(blockIdx.y);
    const int nt = (n_m + kBoxTile - 1) / kBoxTile;
    const int t0x = (sb % nt) * kBoxTile, t0y = ((sb / nt) % nt) * kBoxTile, t0z = (sb / (nt * nt)) * kBoxTile;
    const int64_t K = int64_t(n_m) * n_m * n_m;
    const float half = 0.5f * float(n_m);
    // this thread's sample: a wave covers a 4 x 4 x 4 sub-block of the tile
    // (compact in 3D, which spreads its stencil gathers over more LDS banks
    // than an 8 x 8 x 1 slice)
    const int wq = int(threadIdx.x >> 6), ln = int(threadIdx.x & 63);
    const int i = t0x + 4 * (wq & 1) + (ln & 3), j = t0y + 4 * ((wq >> 1) & 1) + ((ln >> 2) & 3),
              k = t0z + 4 * (wq >> 2) + (ln >> 4);
    const bool ok = i < n_m && j < n_m && k < n_m;
    const int64_t ks = ok ? (int64_t(k) * n_m + j) * n_m + i : 0;
    const float xb0 = float(i) - half, xb1 = float(j) - half, xb2 = float(k) - half;
    const cplx<float> rm = ok ? rho_m[ks] : mk(0.f, 0.f);
    const cplx<float> ck = rm * (ok ? w_m[ks] : 0.f);
    float gw = 0.f, gwi = 0.f;  // wmode 1: Re(rho_M Phi) sum; 2: Phi sum (re, im)
    // body coordinates of the tile corner (a clipped tile keeps the full
    // tile's bounds, which contain its samples)
    const float xlo0 = float(t0x) - half, xlo1 = float(t0y) - half, xlo2 = float(t0z) - half;
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    // staging lane roles: row j_s of a slot of three rows, cell cx_s of the row
    const int js = lane / kBoxRow, cxs = lane - js * kBoxRow;
    const int64_t b0 = int64_t(pb) * kBoxPoses;
    for (int pi = 0; pi < kBoxPoses; ++pi) {
        const int64_t b = b0 + pi;
        if (b >= B) break;  // uniform across the block
        const BoxPose& P = bpose[b];
        float r[9], tfr[3];
        int tint[3], lo[3], ext[3];
#pragma unroll
        for (int a = 0; a < 9; ++a) r[a] = P.r[a];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            tint[a] = P.tint[a];
            tfr[a] = P.tfr[a];
            const float y0 = tfr[a] + r[3 * a] * xlo0 + r[3 * a + 1] * xlo1 + r[3 * a + 2] * xlo2;
            const int fmin = int(floorf(y0 + P.dmin[a] - kBoxMargin));
            lo[a] = __builtin_amdgcn_readfirstlane(fmin - 1 + tint[a]);
            // at most kBoxMax for any rotation (see above); the clamp only guards
            // non-finite poses, whose conversions give in-range but meaningless boxes
            ext[a] = __builtin_amdgcn_readfirstlane(
                min(int(floorf(y0 + P.dmax[a] + kBoxMargin)) - fmin + 4, kBoxMax));
        }
        // stage the box: slot s holds rows 3 q .. 3 q + 2 of plane cz, with
        // s = cz nts + q; lane = kBoxRow j + cx covers row 3 q + j, cell cx
        {
            const unsigned Nu = unsigned(N);
            const unsigned wx = unsigned(wrap(lo[0], N)), wy = __builtin_amdgcn_readfirstlane(wrap(lo[1], N)),
                           wz = __builtin_amdgcn_readfirstlane(wrap(lo[2], N));
            const int nts = (ext[1] + kBoxSlotRows - 1) / kBoxSlotRows, nslot = ext[2] * nts;
            const unsigned inv = 65535u / unsigned(nts) + 1u;  // s / nts = (s inv) >> 16 for s < 2^16 / nts
            unsigned gx = wx + unsigned(cxs);
            gx = min(gx, gx - Nu);
            const bool lane_ok = js < kBoxSlotRows && cxs < ext[0];
            cplx<float> v[kBoxStage];
#pragma unroll
            for (int m = 0; m < kBoxStage; ++m) {
                const int s = wid + m * kBoxWaves;
                v[m] = mk(0.f, 0.f);
                if (s < nslot) {
                    const int cz = int((unsigned(s) * inv) >> 16), q = s - cz * nts;
                    const int cy = q * kBoxSlotRows + js;
                    unsigned gz = wz + unsigned(cz);
                    gz = min(gz, gz - Nu);
                    unsigned gy = wy + unsigned(cy);
                    gy = min(gy, gy - Nu);
                    if (lane_ok && cy < ext[1]) v[m] = rho_f[gz * Nu * Nu + __umul24(gy, Nu) + gx];
                }
            }
#pragma unroll
            for (int m = 0; m < kBoxStage; ++m) {
                const int s = wid + m * kBoxWaves;
                if (s < nslot) {
                    const int cz = int((unsigned(s) * inv) >> 16), q = s - cz * nts;
                    if (lane_ok && q * kBoxSlotRows + js < ext[1])
                        box[cz * kBoxPlane + q * (kBoxSlotRows * kBoxRow) + lane] = v[m];
                }
            }
        }
        __syncthreads();
        const double sc = gscale ? gscale[b] : 1.0;
        double acc[kNAcc];
#pragma unroll
        for (int a = 0; a < kNAcc; ++a) acc[a] = 0.0;
        if (ok) {
            float wgt[3][4], dw[3][4], wv[3];
            int lb[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                wv[a] = r[3 * a] * xb0 + r[3 * a + 1] * xb1 + r[3 * a + 2] * xb2;
                const float y = tfr[a] + wv[a];
                const float fl = floorf(y);
                lb[a] = int(fl) + tint[a] - 1 - lo[a];  // in [0, ext - 4]
                bspline3_weights(y - fl, wgt[a]);
                if (GRAD) bspline3_dweights(y - fl, dw[a]);
            }
            const cplx<float>* base = box + lb[2] * kBoxPlane + lb[1] * kBoxRow + lb[0];
            if constexpr (REAL) {
                // separable contraction of u = Re(c_k v): x, then y, then z
                float phi = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll 1
                for (int cz = 0; cz < 4; ++cz) {
                    float wz = wgt[2][0], dz = dw[2][0];
#pragma unroll
                    for (int q = 1; q < 4; ++q)
                        if (cz == q) {
                            wz = wgt[2][q];
                            dz = dw[2][q];
                        }
                    const cplx<float>* plane = base + cz * kBoxPlane;
                    float ay = 0.f, by = 0.f, cy_ = 0.f;
#pragma unroll
                    for (int cy = 0; cy < 4; ++cy) {
                        float rx = 0.f, rdx = 0.f;
#pragma unroll
                        for (int cx = 0; cx < 4; ++cx) {
                            const cplx<float> v = plane[cy * kBoxRow + cx];
                            const float u = ck.re * v.re - ck.im * v.im;
                            rx += u * wgt[0][cx];
                            rdx += u * dw[0][cx];
                        }
                        ay += rx * wgt[1][cy];
                        by += rdx * wgt[1][cy];
                        cy_ += rx * dw[1][cy];
                    }
                    phi += ay * wz;
                    gx += by * wz;
                    gy += cy_ * wz;
                    gz += ay * dz;
                }
                const double g0 = double(gx), g1 = double(gy), g2 = double(gz);
                const double w0 = double(wv[0]), w1 = double(wv[1]), w2 = double(wv[2]);
                acc[0] = double(phi);
                acc[1] = g0;
                acc[2] = g1;
                acc[3] = g2;
                acc[4] = w1 * g2 - w2 * g1;
                acc[5] = w2 * g0 - w0 * g2;
                acc[6] = w0 * g1 - w1 * g0;
            } else {
                // separable contraction: x, then y, then z
                cplx<float> phi = mk(0.f, 0.f), gx = phi, gy = phi, gz = phi;
#pragma unroll 1
                for (int cz = 0; cz < 4; ++cz) {
                    float wz = wgt[2][0], dz = GRAD ? dw[2][0] : 0.f;
#pragma unroll
                    for (int q = 1; q < 4; ++q)
                        if (cz == q) {
                            wz = wgt[2][q];
                            if (GRAD) dz = dw[2][q];
                        }
                    const cplx<float>* plane = base + cz * kBoxPlane;
                    cplx<float> ay = mk(0.f, 0.f), by = ay, cy_ = ay;
#pragma unroll
                    for (int cy = 0; cy < 4; ++cy) {
                        cplx<float> rx = mk(0.f, 0.f), rdx = rx;
#pragma unroll
                        for (int cx = 0; cx < 4; ++cx) {
                            const cplx<float> v = plane[cy * kBoxRow + cx];
                            rx = rx + v * wgt[0][cx];
                            if (GRAD) rdx = rdx + v * dw[0][cx];
                        }
                        ay = ay + rx * wgt[1][cy];
                        if (GRAD) {
                            by = by + rdx * wgt[1][cy];
                            cy_ = cy_ + rx * dw[1][cy];
                        }
                    }
                    phi = phi + ay * wz;
                    if (GRAD) {
                        gx = gx + by * wz;
                        gy = gy + cy_ * wz;
                        gz = gz + ay * dz;
                    }
                }
                acc[0] = double((ck * phi).re);
                if (GRAD) {
                    const double g0 = double((ck * gx).re), g1 = double((ck * gy).re), g2 = double((ck * gz).re);
                    const double w0 = double(wv[0]), w1 = double(wv[1]), w2 = double(wv[2]);
                    acc[1] = g0;
                    acc[2] = g1;
                    acc[3] = g2;
                    acc[4] = w1 * g2 - w2 * g1;
                    acc[5] = w2 * g0 - w0 * g2;
                    acc[6] = w0 * g1 - w1 * g0;
                    if (want_w == 1) gw += float(sc) * (rm * phi).re;
                    if (want_w == 2) {
                        gw += float(sc) * phi.re;
                        gwi += float(sc) * phi.im;
                    }
                }
            }
        }
        // block reduction: rows of 16 lanes (DPP), then 32 row sums per value
        const int nacc = GRAD ? kNAcc : 1;
#pragma unroll
        for (int a = 0; a < nacc; ++a) {
            const double v = row16_sum(acc[a]);
            if ((lane & 15) == 0) red[wid * 4 + (lane >> 4)][a] = v;
        }
        __syncthreads();  // also: every thread is done reading the box
        if (threadIdx.x < nacc) {
            double v = 0.0;
#pragma unroll
            for (int rw = 0; rw < kBoxBlock / 16; ++rw) v += red[rw][threadIdx.x];
            part[(b * nsb + sb) * kNAcc + threadIdx.x] = v;
        }
    }
    if (GRAD && want_w == 1 && ok) wpart[int64_t(pb) * K + ks] = gw;
    if (GRAD && want_w == 2 && ok) {
        wpart[2 * (int64_t(pb) * K + ks)] = gw;
        wpart[2 * (int64_t(pb) * K + ks) + 1] = gwi;
    }
}

// Per pose: reduce the sample-tile partials, apply the chain rule through
// R(q / |q|) (FP64), write the score and the 7 pose derivatives.
template <typename T, bool GRAD>
__global__ void grad_finish_kernel(const double* __restrict__ part, int nsb, const double* __restrict__ poses,
                                   int64_t B, T* __restrict__ score, double* __restrict__ grad_pose) {
    // one wave per pose: lanes stride over the sample tiles (a pose's partials
    // are contiguous, so a wave's loads are too), then a wave reduction
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    if (b >= B) return;  // uniform across the wave
    double acc[kNAcc];
#pragma unroll
    for (int a = 0; a < kNAcc; ++a) acc[a] = 0.0;
    constexpr int nacc = GRAD ? kNAcc : 1;
    const double* pb = part + b * nsb * kNAcc;
    for (int sb = lane; sb < nsb; sb += 64)
#pragma unroll
        for (int a = 0; a < nacc; ++a) acc[a] += pb[sb * kNAcc + a];
#pragma unroll
    for (int a = 0; a < nacc; ++a) acc[a] = warp_sum(acc[a]);
    if (lane != 0) return;
    score[b] = T(acc[0]);
    if (!GRAD || !grad_pose) return;
    const double* q = poses + 7 * b + 3;
    const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double w = q[0] / nq, x = q[1] / nq, y = q[2] / nq, z = q[3] / nq;
    // df/du_c = 2 vec(e_c u*) . tau (plus a radial part that the projection
    // below removes), u = (w, x, y, z):
    //   vec(1 u*) = (-x, -y, -z), vec(i u*) = (w, z, -y),
    //   vec(j u*) = (-z, w, x),   vec(k u*) = (y, -x, w)
    const double om[4][3] = {{-x, -y, -z}, {w, z, -y}, {-z, w, x}, {y, -x, w}};
    double gu[4];
    for (int c = 0; c < 4; ++c) gu[c] = 2.0 * (om[c][0] * acc[4] + om[c][1] * acc[5] + om[c][2] * acc[6]);
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

// complex tile partials: grad_c[k] = sum over pose tiles of Phi sums
template <typename T>
__global__ void csum_kernel(const T* __restrict__ wpart, int npb, int64_t K, T* __restrict__ grad_c) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= K) return;
    T re = T(0), im = T(0);
    for (int p = 0; p < npb; ++p) {
        re += wpart[2 * (int64_t(p) * K + k)];
        im += wpart[2 * (int64_t(p) * K + k) + 1];
    }
    grad_c[2 * k] = re;
    grad_c[2 * k + 1] = im;
}

// grad_w[k] = Re(rho_M[k] grad_c[k])
template <typename T>
__global__ void w_from_c_kernel(const cplx<T>* __restrict__ rho_m, const T* __restrict__ grad_c, int64_t K,
                                T* __restrict__ grad_w) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= K) return;
    grad_w[k] = rho_m[k].re * grad_c[2 * k] - rho_m[k].im * grad_c[2 * k + 1];
}

// ---- chain-rule products for automatic differentiation
// out[b][j] = gp[b][j] * s[b] (FP64; may be in place)
__global__ void pose_chain_kernel(const double* __restrict__ gp, const double* __restrict__ s, int64_t B,
                                  double* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= 7 * B) return;
    out[i] = gp[i] * s[i / 7];
}

// cotangent of rho_M from that of c_k = w_k rho_M(x_k): w_k G_k (complex)
template <typename T>
__global__ void rho_from_c_kernel(const T* __restrict__ w_m, const T* __restrict__ grad_c, int64_t K,
                                  T* __restrict__ grad_rho) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= K) return;
    grad_rho[2 * k] = w_m[k] * grad_c[2 * k];
    grad_rho[2 * k + 1] = w_m[k] * grad_c[2 * k + 1];
}

// zero `count` values of type T (a kernel rather than hipMemsetAsync, so that
// the calls stay valid inside captured graphs)
template <typename T>
__global__ void zero_fill_kernel(T* __restrict__ p, int64_t count) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = T(0);
}

// ---- cotangent of the scores with respect to rho_F (the adjoint of the
// gather): G(p) = sum_b s_b sum_k c_k B3(p - y_kb), periodic, y_kb = R_b x_k + t_b.
// Per pose: R (FP64) and t split into floor and fraction, so that positions
// are formed near the origin in T.
__global__ void fixed_pose_kernel(const double* __restrict__ poses, int64_t B, double* __restrict__ out) {
    const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double* pose = poses + 7 * b;
    double r[9];
    quat_rot(pose + 3, r);
#pragma unroll
    for (int a = 0; a < 9; ++a) out[12 * b + a] = r[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) out[12 * b + 9 + a] = pose[a];
}

// One thread per (body node, pose): the node's coefficient times s_b, spread
// with its 4^3 (planar 4^2) B-spline stencil by atomic adds.
template <typename T>
__global__ void fixed_cot_kernel(const cplx<T>* __restrict__ rho_m, const T* __restrict__ w_m, int n_m, int planar,
                                 const double* __restrict__ pr, const double* __restrict__ gscale, int64_t B,
                                 int b0, int N, T* __restrict__ out) {
    const int64_t K = planar ? int64_t(n_m) * n_m : int64_t(n_m) * n_m * n_m;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t b = b0 + int64_t(blockIdx.y);
    if (k >= K || b >= B) return;
    const T sb = T(gscale ? gscale[b] : 1.0);
    const cplx<T> ck = rho_m[k] * (w_m[k] * sb);
    if (ck.re == T(0) && ck.im == T(0)) return;
    const double* P = pr + 12 * b;
    const T half = T(0.5) * T(n_m);
    const T xb[3] = {T(int(k % n_m)) - half, T(int((k / n_m) % n_m)) - half,
                     planar ? T(0) : T(int(k / (int64_t(n_m) * n_m))) - half};
    int base[3];
    T wgt[3][4];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double ti = floor(P[9 + a]);
        const T y = T(P[9 + a] - ti) + T(P[3 * a]) * xb[0] + T(P[3 * a + 1]) * xb[1] + T(P[3 * a + 2]) * xb[2];
        const T fl = dev_floor(y);
        base[a] = int(fl) + int(ti) - 1;
        bspline3_weights(y - fl, wgt[a]);
    }
    const int zc = planar ? 1 : 4;
    for (int cz = 0; cz < zc; ++cz) {
        const int iz = planar ? 0 : wrap(base[2] + cz, N);
        const T wz = planar ? T(1) : wgt[2][cz];
        for (int cy = 0; cy < 4; ++cy) {
            const int iy = wrap(base[1] + cy, N);
            const T wyz = wgt[1][cy] * wz;
            for (int cx = 0; cx < 4; ++cx) {
                const int ix = wrap(base[0] + cx, N);
                const T wt = wgt[0][cx] * wyz;
                const int64_t idx = (int64_t(iz) * N + iy) * N + ix;
                atomicAdd(out + 2 * idx, ck.re * wt);
                atomicAdd(out + 2 * idx + 1, ck.im * wt);
            }
        }
    }
}

}  // namespace

// the LDS-staged kernel serves 3D FP32 poses; FP64 and planar use the tile kernel
template <typename T>
bool use_box(bool planar, int N) {
    return std::is_same<T, float>::value && !planar && N >= kBoxMax && N <= 1024;
}

template <typename T>
void grad_tiles(int64_t B, int N, int n_m, bool planar, int64_t* nsb, int64_t* npb) {
    const int64_t K = planar ? int64_t(n_m) * n_m : int64_t(n_m) * n_m * n_m;
    if (use_box<T>(planar, N)) {
        const int64_t nt = (n_m + kBoxTile - 1) / kBoxTile;
        *nsb = nt * nt * nt;
        *npb = (B + kBoxPoses - 1) / kBoxPoses;
    } else {
        *nsb = (K + kSamplesPerBlock - 1) / kSamplesPerBlock;
        *npb = (B + kPosesPerBlock - 1) / kPosesPerBlock;
    }
}

template <typename T>
size_t grad_workspace_bytes(int64_t B, int N, int n_m, bool planar, int wmode) {
    const int64_t K = planar ? int64_t(n_m) * n_m : int64_t(n_m) * n_m * n_m;
    int64_t nsb, npb;
    grad_tiles<T>(B, N, n_m, planar, &nsb, &npb);
    size_t bytes = size_t(B * nsb * kNAcc) * sizeof(double);
    bytes = (bytes + 255) / 256 * 256;
    if (wmode) bytes += (size_t(npb * K) * sizeof(T) * size_t(wmode) + 255) / 256 * 256;
    if (use_box<T>(planar, N)) bytes += size_t(B) * sizeof(BoxPose);
    return bytes + 256;
}

template <typename T>
hipError_t launch_score_grad(const void* rho_f, int N, bool planar, const void* rho_m, const T* w_m, int n_m,
                             const double* poses, int64_t B, T* score, double* grad_pose, T* grad_w, T* grad_c,
                             const double* grad_scale, void* ws, hipStream_t s) {
    const int64_t K = planar ? int64_t(n_m) * n_m : int64_t(n_m) * n_m * n_m;
    int64_t nsb64, npb64;
    grad_tiles<T>(B, N, n_m, planar, &nsb64, &npb64);
    const int nsb = int(nsb64), npb = int(npb64);
    double* part = static_cast<double*>(ws);
    size_t off = size_t(B * nsb * kNAcc) * sizeof(double);
    off = (off + 255) / 256 * 256;
    T* wpart = reinterpret_cast<T*>(static_cast<char*>(ws) + off);
    // weight mode: 2 sums Phi (complex) per sample, from which grad_w follows;
    // 1 sums Re(rho_M Phi) directly
    const int ww = grad_c ? 2 : (grad_w ? 1 : 0);
    if (ww) off += (size_t(npb64 * K) * sizeof(T) * size_t(ww) + 255) / 256 * 256;
    BoxPose* bpose = reinterpret_cast<BoxPose*>(static_cast<char*>(ws) + off);
    if (use_box<T>(planar, N)) {
        hipLaunchKernelGGL(box_pose_kernel, dim3(unsigned((B + 127) / 128)), dim3(128), 0, s, poses, B, bpose);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const bool grad = grad_pose != nullptr || ww != 0;
    const auto* rf = static_cast<const cplx<T>*>(rho_f);
    const auto* rm = static_cast<const cplx<T>*>(rho_m);
    // pose tiles run in launches of at most 65535 along grid y
    for (int pb0 = 0; pb0 < npb; pb0 += 65535) {
        const dim3 grid{unsigned(nsb), unsigned(std::min(npb - pb0, 65535)), 1u};
        if constexpr (std::is_same<T, float>::value) {
            if (use_box<T>(planar, N)) {
                if (grad && ww == 0)
                    hipLaunchKernelGGL((grad_box_kernel<true, true>), grid, dim3(kBoxBlock), 0, s, rf, N, rm, w_m, n_m,
                                       bpose, B, grad_scale, part, nsb, wpart, 0, pb0);
                else if (grad)
                    hipLaunchKernelGGL((grad_box_kernel<true>), grid, dim3(kBoxBlock), 0, s, rf, N, rm, w_m, n_m, bpose,
                                       B, grad_scale, part, nsb, wpart, ww, pb0);
                else
                    hipLaunchKernelGGL((grad_box_kernel<false>), grid, dim3(kBoxBlock), 0, s, rf, N, rm, w_m, n_m,
                                       bpose, B, grad_scale, part, nsb, wpart, 0, pb0);
            }
        }
        if (!use_box<T>(planar, N)) {
            if (grad)
                hipLaunchKernelGGL((grad_tile_kernel<T, true>), grid, dim3(kGBlock), 0, s, rf, N, planar ? 1 : 0, rm,
                                   w_m, n_m, poses, B, grad_scale, part, nsb, wpart, ww, pb0);
            else
                hipLaunchKernelGGL((grad_tile_kernel<T, false>), grid, dim3(kGBlock), 0, s, rf, N, planar ? 1 : 0, rm,
                                   w_m, n_m, poses, B, grad_scale, part, nsb, wpart, 0, pb0);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 g2(unsigned((B + 3) / 4));  // 4 waves of 64 lanes per block, one pose per wave
    if (grad)
        hipLaunchKernelGGL((grad_finish_kernel<T, true>), g2, dim3(256), 0, s, part, nsb, poses, B, score, grad_pose);
    else
        hipLaunchKernelGGL((grad_finish_kernel<T, false>), g2, dim3(256), 0, s, part, nsb, poses, B, score, nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 gk(unsigned((K + 255) / 256));
    if (ww == 1) {
        hipLaunchKernelGGL(wsum_kernel<T>, gk, dim3(256), 0, s, wpart, npb, K, grad_w);
    } else if (ww == 2) {
        hipLaunchKernelGGL(csum_kernel<T>, gk, dim3(256), 0, s, wpart, npb, K, grad_c);
        if (grad_w) hipLaunchKernelGGL(w_from_c_kernel<T>, gk, dim3(256), 0, s, rm, grad_c, K, grad_w);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fixed_cotangent(const void* rho_m, const T* w_m, int n_m, bool planar, int N, const double* poses,
                                  int64_t B, const double* grad_scale, void* grad_f, void* ws, hipStream_t s) {
    const int64_t K = planar ? int64_t(n_m) * n_m : int64_t(n_m) * n_m * n_m;
    const int64_t G = planar ? int64_t(N) * N : int64_t(N) * N * N;
    hipLaunchKernelGGL(zero_fill_kernel<T>, dim3(unsigned(std::min<int64_t>((2 * G + 255) / 256, 4096))), dim3(256), 0,
                       s, static_cast<T*>(grad_f), 2 * G);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    double* pr = static_cast<double*>(ws);
    hipLaunchKernelGGL(fixed_pose_kernel, dim3(unsigned((B + 127) / 128)), dim3(128), 0, s, poses, B, pr);
    for (int64_t b0 = 0; b0 < B; b0 += 65535) {
        const dim3 grid{unsigned((K + 255) / 256), unsigned(std::min<int64_t>(B - b0, 65535)), 1u};
        hipLaunchKernelGGL(fixed_cot_kernel<T>, grid, dim3(256), 0, s, static_cast<const cplx<T>*>(rho_m), w_m, n_m,
                           planar ? 1 : 0, pr, grad_scale, B, int(b0), N, static_cast<T*>(grad_f));
    }
    return hipGetLastError();
}

hipError_t launch_pose_chain(const double* gp, const double* scale, int64_t B, double* out, hipStream_t s) {
    hipLaunchKernelGGL(pose_chain_kernel, dim3(unsigned((7 * B + 255) / 256)), dim3(256), 0, s, gp, scale, B, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rho_from_c(const T* w_m, const void* grad_c, int64_t K, void* grad_rho, hipStream_t s) {
    hipLaunchKernelGGL(rho_from_c_kernel<T>, dim3(unsigned((K + 255) / 256)), dim3(256), 0, s, w_m,
                       static_cast<const T*>(grad_c), K, static_cast<T*>(grad_rho));
    return hipGetLastError();
}
template hipError_t launch_rho_from_c<float>(const float*, const void*, int64_t, void*, hipStream_t);
template hipError_t launch_rho_from_c<double>(const double*, const void*, int64_t, void*, hipStream_t);

hipError_t launch_zero_f64(double* p, int64_t count, hipStream_t s) {
    hipLaunchKernelGGL(zero_fill_kernel<double>, dim3(unsigned(std::min<int64_t>((count + 255) / 256, 4096))),
                       dim3(256), 0, s, p, count);
    return hipGetLastError();
}

template hipError_t launch_fixed_cotangent<float>(const void*, const float*, int, bool, int, const double*, int64_t,
                                                  const double*, void*, void*, hipStream_t);
template hipError_t launch_fixed_cotangent<double>(const void*, const double*, int, bool, int, const double*, int64_t,
                                                   const double*, void*, void*, hipStream_t);
template size_t grad_workspace_bytes<float>(int64_t, int, int, bool, int);
template size_t grad_workspace_bytes<double>(int64_t, int, int, bool, int);
template hipError_t launch_score_grad<float>(const void*, int, bool, const void*, const float*, int, const double*,
                                             int64_t, float*, double*, float*, float*, const double*, void*,
                                             hipStream_t);
template hipError_t launch_score_grad<double>(const void*, int, bool, const void*, const double*, int, const double*,
                                              int64_t, double*, double*, double*, double*, const double*, void*,
                                              hipStream_t);

}  // namespace sdf
