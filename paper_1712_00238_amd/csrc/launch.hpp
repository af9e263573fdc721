// Host-side launchers of the sdfdock kernels.  Every launcher enqueues on
// `stream` and returns the launch status (hipGetLastError after the
// launch); shapes are validated by the ABI layer before any launcher runs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sdf {

struct GridDesc {
    int nx, ny, nz;
    double ox, oy, oz, h;
};
struct ParamDesc {
    double lambda1, lambda2, sigma, eps, xi_floor;
};

// ---- skeletal density (sdf_build)
template <typename T>
hipError_t launch_sdf_build(const T* q, const T* n, const T* w, int64_t ns, const GridDesc& g,
                            const ParamDesc& p, void* rho_out, hipStream_t s);

// ---- rotations: quaternions (FP64, device) -> R (FP64 and cast to T), n x 9 row-major
template <typename T>
hipError_t launch_quat_to_rot(const double* quats, int64_t n, double* r64, T* rT, hipStream_t s);

// ---- per-sample coefficients c_k = w_k rho_M(x_k)
template <typename T>
hipError_t launch_coef(const void* rho_m, const T* w_m, int64_t count, void* c_out, hipStream_t s);

// ---- plain multi-pass path (any T)
// zero `count` complex values
template <typename T>
hipError_t launch_zero(void* buf, int64_t count, hipStream_t s);
// spread samples c (n_m^3 or n_m^2) rotated by R[rot] (sign * R x_k) into grids
// out[rot], which must be zero.  n_rot rotations, R in T.
template <typename T>
hipError_t launch_spread_atomic(const void* c, int n_m, bool planar, const T* R, int n_rot, T sign, int N,
                                void* out, hipStream_t s);
// in-place 3D (or 2D) FFT of `batch` N^3 (N^2) grids; dir -1 forward, +1 inverse;
// results multiplied by `scale`.
template <typename T>
hipError_t launch_fft3(void* data, int N, bool planar, int batch, int dir, double scale, hipStream_t s);
// data[b] *= spec, elementwise, batch grids of `count`
template <typename T>
hipError_t launch_mul_spec(void* data, const void* spec, int64_t count, int batch, hipStream_t s);
// per-rotation peak from complex volumes (Re part) or real volumes.
// partial: per block (value, index); final writes score, t, nbhd, refined.
template <typename T>
hipError_t launch_peak(const void* vol, bool vol_is_complex, int N, bool planar, int batch, T* part_val,
                       int* part_idx, int nparts, T* score, int32_t* t, T* nbhd, double* refined,
                       hipStream_t s);
template <typename T>
int peak_parts(int N, bool planar);
// real part of complex volumes into real output
template <typename T>
hipError_t launch_real_part(const void* vol, T* out, int64_t count, hipStream_t s);

// Optional per-kernel timing hook: begin/end bracket one kernel launch on a
// stream (implemented with HIP events by the ABI layer).
struct KernelTimer {
    virtual void begin(const char* name, hipStream_t s) = 0;
    virtual void end(hipStream_t s) = 0;
    virtual ~KernelTimer() = default;
};

// ---- fused FP32 path
struct FusedPlan {
    int N;
    int n_m;
    bool planar;
    int batch;        // rotations per batch (even)
    int pencil_group; // rotations per pencil job (2 or 4)
};
size_t fused_workspace_bytes(const FusedPlan& fp);
// once per search call, after the coefficients and before the batches
hipError_t launch_fused_prep(const FusedPlan& fp, const void* c, void* ws, hipStream_t s);
// score `n_rot` (<= batch) rotations whose FP32 matrices are R (device, n_rot x 9)
hipError_t launch_fused_batch(const FusedPlan& fp, const float* R, int n_rot, const void* c, const void* spec,
                              void* ws, float* score, int32_t* t, float* nbhd, double* refined, hipStream_t s,
                              KernelTimer* kt = nullptr);

// ---- top-k
template <typename T>
hipError_t launch_topk(const T* scores, int64_t n, int64_t k, void* ws, int32_t* idx_out, hipStream_t s);
size_t topk_workspace_bytes(int64_t n);

// ---- score_grad
template <typename T>
size_t grad_workspace_bytes(int64_t B, int n_m, bool planar, bool want_w);
template <typename T>
hipError_t launch_score_grad(const void* rho_f, int N, bool planar, const void* rho_m, const T* w_m, int n_m,
                             const double* poses, int64_t B, T* score, double* grad_pose, T* grad_w,
                             const double* grad_scale, void* ws, hipStream_t s);

}  // namespace sdf
