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
    double radius = 0.0;  // probe radius R of the radial-basis and double-skin-layer kernels
};

// kernels of eq. 13 (the values of sdf_phi_kind)
constexpr int kPhiSkeletal = 0, kPhiInverseSquare = 1, kPhiRadial = 2, kPhiDsl = 3;

// ---- skeletal density (sdf_build): FP64 samples, output in T
size_t sdf_build_workspace_bytes(int64_t ns, int phi = kPhiSkeletal);
// stats (may be null; skeletal kernel only): three device counters that the
// build adds its pass-1 pairs, pass-2 pairs and in-ball pairs to
template <typename T>
hipError_t launch_sdf_build(const double* q, const double* n, const double* w, int64_t ns, const GridDesc& g,
                            const ParamDesc& p, int phi, void* rho_out, void* ws, hipStream_t s,
                            unsigned long long* stats = nullptr);
// adjoint of sdf_build: gradients (FP64, zeroed here) of Re sum_p cot(p) rho(p)
// with respect to the sample positions, normals and weights
template <typename T>
hipError_t launch_sdf_adjoint(const double* q, const double* n, const double* w, int64_t ns, const GridDesc& g,
                              const ParamDesc& p, const void* cot, double* grad_q, double* grad_n, double* grad_w,
                              void* ws, hipStream_t s);

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
// direct reference: boundary samples turned about c (FP64), and body-box
// values placed on the fixed grid at the reflected integer offsets
hipError_t launch_rotate_samples(const double* q, const double* nrm, int64_t ns, const double* R, const double c[3],
                                 double* qo, double* no, hipStream_t s);
template <typename T>
hipError_t launch_place_direct(const void* rho, int n_m, bool planar, T w_node, int N, void* out, hipStream_t s);
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
// Per-kernel timing: the timer hands out a start / stop event pair that the
// kernel's own dispatch records (hipExtLaunchKernelGGL), so the interval is
// the kernel's execution, as a kernel trace reports it.
struct KernelTimer {
    virtual void events(const char* name, hipEvent_t* start, hipEvent_t* stop) = 0;
    virtual ~KernelTimer() = default;
};

// ---- fused FP32 path
// One pair of a (possibly multi-pair) search, device-resident.
struct FusedJob {
    const void* c;       // complex64 coefficients c_k = w_k rho_M(x_k), n_m^3 (n_m^2 planar)
    const void* spec;    // complex64 fixed spectrum
    float* scale;        // [fixed-point scale, its inverse], written by the prep kernels
    float* score;        // per-rotation outputs of this pair
    int32_t* t;
    float* nbhd;         // may be null
    double* refined;     // may be null
    int n_m;
    int planar;          // 1: n_m^2 x 1 body box
};
// One rotation of the search, device-resident: FP32 matrix, owning pair,
// index of the rotation within that pair's outputs, and the range of centred
// slab heights [zlo, zhi] that the rotated body box can reach (slabs outside
// it are identically zero: the spread kernel does not write them and the
// pencil kernel reads zeros instead).
struct FusedRot {
    float R[9];
    int job;
    int local;
    short zlo, zhi;
};
// Host-side input of one rotation: FP64 quaternion, pair, local index, and
// the body box and grid sizes that bound its slab range.
struct RotInput {
    double q[4];
    int job;
    int local;
    int n_m;
    int N;      // fixed grid size; 0 for a planar pair (one slab, always reached)
};
struct FusedPlan {
    int N;
    bool planar;
    int batch;         // rotations per batch
    int pencil_group;  // rotations per pencil block (2 or 4)
    int radix;         // radix schedule variant (0, 1, 2)
    int max_wgs;       // persistent grid size cap (0 = one work item per block)
};
size_t fused_workspace_bytes(const FusedPlan& fp);
// occupancy of the fused kernels, queried once per process (the context's
// creation calls it, before any launch sequence can be captured)
void fused_query_occupancy();
// 3D grids of N = 64 and 128 pass grids between the fused kernels with their
// x columns in pair-grouped order (each aligned block of 16 positions holds
// 8 columns kx and their negatives); the spread slabs go from the spread to
// the pencil pass in column tiles (one row ky, one block of 16 positions,
// every kz), and the fixed spectrum is copied into that order and tiling
// once per call.
inline bool fused_pair_grouped(int N, bool planar) { return !planar && (N == 64 || N == 128); }
hipError_t launch_spec_pair_group(const void* spec, void* out, int N, hipStream_t s);
// quaternions -> FusedRot descriptors (FP64 matrix, cast to FP32)
hipError_t launch_rot_desc(const RotInput* in, int64_t n, FusedRot* out, hipStream_t s);
// per pair: max |c_k| and the fixed-point scale (written through jobs[j].scale)
hipError_t launch_fused_prep(const FusedJob* jobs, int n_jobs, void* scratch, hipStream_t s);
size_t fused_prep_scratch_bytes(int n_jobs);
// score rotations rots[0 .. n_rot) (n_rot <= fp.batch) of one grid-size class
hipError_t launch_fused_batch(const FusedPlan& fp, const FusedRot* rots, int n_rot, const FusedJob* jobs, void* ws,
                              hipStream_t s, KernelTimer* kt = nullptr);
// Peaks of rotations whose correlation spectra Y(k) S(k) are already formed
// (complex64, 3D, N = 64 or 128, nb grids in column tiles with pair-grouped
// positions, as launch_nfft_modes writes them with `tiled`): fold rotation
// pairs, inverse FFT through the search path's pencil, inverse-slab and finish
// kernels, outputs as score_rotations for rotation i at index i.
bool modes_peaks_supported(int N, bool planar);
size_t modes_peaks_workspace_bytes(int N, int nb);
hipError_t launch_modes_peaks(int N, const void* modes, int nb, int n_m, float* score, int32_t* t, float* nbhd,
                              double* refined, int num_cu, void* ws, hipStream_t s);
// deterministic pseudo-random complex64 fill (autotune inputs)
hipError_t launch_fill_random(void* data, int64_t count, uint32_t seed, float amp, hipStream_t s);

// ---- nonequispaced route: octree-adaptive samples and the type-1 transform
// workspace of launch_octree for an N_M box of `elem`-byte reals
size_t octree_workspace_bytes(int nm, bool planar, size_t elem);
// leaves of the adaptive tree over c = w rho_M (N_M % 8 == 0, max_level <= 3):
// pos (3 per leaf, grid units from the body origin), c_out, level (may be
// NULL) in block / Morton order; *count_out (device) = number of leaves
template <typename T>
hipError_t launch_octree(const void* rho_m, const T* w_m, int nm, bool planar, double tol, int max_level, T* pos,
                         void* c_out, int* level, int64_t* count_out, void* ws, hipStream_t s);
// 1 / phihat of the width-w kernel for the N FFT-order modes of the 2N grid
template <typename T>
hipError_t launch_es_deconv(int N, int w, T* inv, hipStream_t s);
// `batch` rotations R[b] (9 T each) of the m samples: bin them per tile of
// the (2N)^d grids `fine`, spread tile by tile (every node written),
// transform, and write out[b] = deconvolved N^d modes times spec (ready for
// the inverse FFT of the correlation); ws holds nfft_workspace_bytes
size_t nfft_workspace_bytes(int64_t m, int batch, int N, bool planar, size_t elem);
// per rotation: bytes of the `fine` grid launch_nfft_modes needs (the whole
// (2N)^d grid, or a quarter of it where the x pass is fused into the tiles)
size_t nfft_grid_bytes(int N, bool planar, size_t elem);
// tiled (3D, N = 64 or 128): out in column tiles with pair-grouped positions
// (the input of launch_modes_peaks) instead of [b][jz][jy][jx]
template <typename T>
hipError_t launch_nfft_modes(const T* pos, const void* c, int64_t m, const T* R, int batch, int N, bool planar,
                             int w, const T* inv, const void* spec, void* fine, void* out, void* ws, hipStream_t s,
                             bool tiled = false);

// ---- exclusive prefix sum of n ints (out may not alias in); temp holds
// scan_temp_bytes(n)
size_t scan_temp_bytes(int64_t n);
hipError_t launch_exclusive_scan(const int* in, int* out, int64_t n, void* temp, hipStream_t s);
// ---- stable sort of (key, value) pairs by the low `bits` bits of the keys,
// least-significant digit first over 8-bit digits, ping-ponging between the
// given buffers; *keys_sorted / *vals_sorted name the buffers holding the
// result.  temp holds sort_temp_bytes(n).
size_t sort_temp_bytes(int64_t n);
hipError_t launch_sort_pairs(unsigned* keys, int* vals, unsigned* keys_alt, int* vals_alt, int64_t n, int bits,
                             void* temp, hipStream_t s, unsigned** keys_sorted, int** vals_sorted);

// ---- top-k
template <typename T>
hipError_t launch_topk(const T* scores, int64_t n, int64_t k, void* ws, int32_t* idx_out, hipStream_t s);
size_t topk_workspace_bytes(int64_t n);

// ---- score_grad
template <typename T>
size_t grad_workspace_bytes(int64_t B, int N, int n_m, bool planar, int wmode);
// grad_c (may be NULL): complex per-sample sums of grad_scale_b Phi_b(y_k);
// grad_w then follows as Re(rho_M grad_c)
// cotangent of sum_b s_b f_b with respect to rho_F (complex, zeroed here);
// ws: 12 B doubles
template <typename T>
hipError_t launch_fixed_cotangent(const void* rho_m, const T* w_m, int n_m, bool planar, int N, const double* poses,
                                  int64_t B, const double* grad_scale, void* grad_f, void* ws, hipStream_t s);
// out[b][j] = gp[b][j] * scale[b], FP64 B x 7 (may be in place)
hipError_t launch_pose_chain(const double* gp, const double* scale, int64_t B, double* out, hipStream_t s);
// grad_rho[k] = w_m[k] grad_c[k] (complex, context precision)
template <typename T>
hipError_t launch_rho_from_c(const T* w_m, const void* grad_c, int64_t K, void* grad_rho, hipStream_t s);
// zero `count` doubles with a kernel (valid inside captured graphs)
hipError_t launch_zero_f64(double* p, int64_t count, hipStream_t s);
template <typename T>
hipError_t launch_score_grad(const void* rho_f, int N, bool planar, const void* rho_m, const T* w_m, int n_m,
                             const double* poses, int64_t B, T* score, double* grad_pose, T* grad_w, T* grad_c,
                             const double* grad_scale, void* ws, hipStream_t s);

}  // namespace sdf
