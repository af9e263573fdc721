/*
 * sdfdock.h - C ABI of the MI355X (gfx950) shape-complementarity scoring
 * library: skeletal density functions (SDFs) of two solids and the
 * cross-correlation score over rigid placements, after Behandish & Ilies,
 * "Shape Complementarity Analysis for Objects of Arbitrary Shape"
 * (tech. report CDL-TR-14-01, 2014; arXiv 1712.00238).
 *
 * The paper poses the problem as: given a fixed solid S1 and a moving solid
 * S2, score every relative placement tau in SE(3) by
 *     f(tau) = integral rho_1(p) rho_2(tau^-1 p) dv                 (eq. 8)
 * where rho is the skeletal density function of eq. 13 / 15 / 16c / 17t,
 * and return the placements with the highest scores (Formulation section).
 * Rigid motions are split into a rotation set times all grid translations,
 * and each rotation's translations are scored at once through FFTs
 * (Implementation section).
 *
 * Conventions used by every call
 * ------------------------------
 *  - Memory: every array argument is a caller-owned DEVICE pointer unless
 *    marked (host).  The library never frees or retains caller memory.
 *    Device arrays must be 16-byte aligned (any allocation from hipMalloc or
 *    PyTorch qualifies).
 *  - Precision: a context has a dtype.  SDF_F32 contexts take and return
 *    float (real) / float2 (complex) arrays, SDF_F64 contexts double /
 *    double2.  "real" and "complex" below mean the context's type.  Rotation
 *    matrices, sub-voxel offsets and pose gradients are computed in FP64 in
 *    both precisions.
 *  - Complex arrays are interleaved (re, im).
 *  - Grids: sdf_grid.n = (nx, ny, nz) nodes, node (i, j, k) at world
 *    origin + h * (i, j, k); arrays are [k][j][i] with i fastest, flat index
 *    (k * ny + j) * nx + i.  Planar (2D) work uses nz = 1, samples with
 *    z = 0 and in-plane normals, rotations about +z.
 *  - Moving body box: a grid of N_M^3 (or N_M^2 x 1) nodes whose node k sits
 *    at body position x_k = h (k - N_M / 2) relative to the body origin;
 *    g_moving.origin is the world position of node 0 in the moving part's
 *    own frame (body origin - h N_M / 2).
 *  - Pose (R, t): the body point x goes to R x + o_F + h t, with o_F the
 *    fixed grid origin and t in grid units.  Scores of integer t are
 *        f(R, t) = Re sum_p rho_F(p) M_R((p - t) mod N),
 *        M_R(u)  = sum_k c_k B3(u - R x_k / h),  c_k = w_k rho_M(x_k),
 *    B3 the tensor cubic B-spline (the grid is periodic).
 *  - Quaternions are (w, x, y, z), Hamilton convention, R = R(q / |q|).
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream).  A context is not thread-safe: use one per thread / stream.
 *  - Return value: SDF_OK (0) or a negative error code.  On error nothing
 *    was enqueued, inputs are untouched, outputs are unspecified and
 *    sdf_last_error() holds a message.  Faults inside kernels surface at the
 *    caller's next synchronisation.  No C++ exception crosses the ABI.
 */
#ifndef SDFDOCK_H
#define SDFDOCK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sdf_ctx_s *sdf_ctx;
typedef void *sdf_stream; /* a hipStream_t */

typedef enum { SDF_F32 = 0, SDF_F64 = 1 } sdf_dtype;

enum {
    SDF_OK = 0,
    SDF_EINVAL = -1,       /* null pointer, bad size / shape, non-finite parameter, zero quaternion */
    SDF_EUNSUPPORTED = -2, /* FFT size outside {8, 16, 32, 64, 96, 128}, dtype / device mismatch */
    SDF_EHIP = -3,         /* HIP runtime error while enqueueing */
    SDF_ENOMEM = -4        /* workspace would exceed the context's cap, or allocation failed */
};

typedef struct {
    int32_t n[3];      /* nodes per axis (x, y, z); n[2] = 1 for planar work */
    double origin[3];  /* world position of node (0, 0, 0) */
    double h;          /* node spacing (> 0); both parts of a pair use the same h */
} sdf_grid;

/* Affinity parameters (eq. 15 / 16c / 17t): lambda1 > 0 weights exterior
 * points, lambda2 > 0 interior points, sigma > 0 is the thickness factor,
 * eps >= 0 the truncation factor of the contact region, xi_floor >= 0 the
 * distance below which a node counts as on the boundary (rho := 0 there).
 * The planar validation runs use lambda1 = 1, lambda2 = 3, sigma = 0.5,
 * eps = 1.5. */
typedef struct {
    double lambda1, lambda2, sigma, eps, xi_floor;
} sdf_params;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  `workspace_cap_bytes` bounds the
 * device workspace the context may hold (0 = no cap).  Workspace grows
 * lazily on the first call that needs it and is reused afterwards.
 * Errors: SDF_EINVAL (out == NULL, bad dtype), SDF_EHIP (no such device). */
int sdf_ctx_create(sdf_ctx *out, int device, sdf_dtype dtype, size_t workspace_cap_bytes);

/* Release the workspace, cached plans and graphs.  Synchronises the device
 * first.  NULL is ignored. */
void sdf_ctx_destroy(sdf_ctx ctx);

/* Message of the last failing call on `ctx` (or of the last failing call
 * on this thread when ctx is NULL).  Valid until the next call. */
const char *sdf_last_error(sdf_ctx ctx);

/* Tuning options (integers):
 *   "path"          0 auto, 1 plain multi-pass kernels, 2 fused kernels (F32 only)
 *   "batch"         rotations per fused launch sequence (even, 2..256; default 64)
 *   "graph"         1: capture each batch's launch sequence in a hipGraph and replay it
 *   "pencil_group"  rotations sharing one spectrum tile in the fused pencil pass (2 or 4)
 *   "profile"       1: time every fused kernel (see sdf_ctx_stats)
 *   "radix"         FFT radix schedule of the fused kernels for N = 8, 16, 32, 96 (0, 1, 2;
 *                   e.g. 96 = 8.4.3, 3.4.8, 4.8.3); N = 64 and 128 use fixed two-pass transforms
 *   "autotune"      1: tune each grid-size class on its first search (see sdf_autotune)
 *   "autotune_reject" bit i set: the autotuner treats its i-th candidate (in the order
 *                   batch, then group, then schedule, as in its report) as failing the
 *                   parity probe (for testing the failure path; default 0)
 *   "sdf_stats"     1: sdf_build (skeletal kernel) runs a counting variant that adds its
 *                   node-sample pairs to three counters (setting the option clears them):
 *                   "sdf_pairs_nearest" (pass 1: valid nodes x samples of the tiles
 *                   visited for the nearest sample), "sdf_pairs_sum" (pass 2: live nodes x
 *                   samples of the tiles visited for the kernel sum) and "sdf_pairs_in_ball"
 *                   (pairs inside the contact ball), read with sdf_ctx_get_option (which
 *                   synchronises the device).  For measurement, not for timed builds.
 * With "graph" = 1 the fused launch sequence of a score_rotations call is
 * captured once and replayed while the buffers, shapes and stream stay the
 * same; the null stream cannot be captured and runs without a graph.
 * Errors: SDF_EINVAL for an unknown key or out-of-range value. */
int sdf_ctx_set_option(sdf_ctx ctx, const char *key, int64_t value);
/* Read an option, the device's compute-unit count "num_cu", or one of the
 * counters "graph_captures", "graph_launches", "sdf_pairs_nearest",
 * "sdf_pairs_sum", "sdf_pairs_in_ball". */
int sdf_ctx_get_option(sdf_ctx ctx, const char *key, int64_t *value);

/* Kernel timing.  With the option "profile" = 1 every kernel of the fused
 * search is launched with a start / stop HIP event pair that its own
 * dispatch records (the kernel's execution interval; graphs are not used
 * meanwhile).  sdf_ctx_stats synchronises on the recorded events and returns
 * the accumulated time and launch count of one kernel ("spread_slab",
 * "pencil", "islab_peak", "finish", "finish_rot"; unknown names give 0).
 * sdf_ctx_stats_reset clears the totals. */
int sdf_ctx_stats(sdf_ctx ctx, const char *kernel, double *total_ms, int64_t *launches);
int sdf_ctx_stats_reset(sdf_ctx ctx);

/* ------------------------------------------------------- skeletal density */

/* Skeletal density function of one solid on a grid (eq. 10A, 11, 12a, 13,
 * 15, 16c, 17t), by point quadrature over oriented boundary samples:
 *   xi_abs = min_j |p - q_j|, j* its lowest-index minimiser,
 *   pmc    = sign((p - q_j*) . n_j*),
 *   rho(p) = 0 if pmc = 0 or xi_abs < xi_floor, else
 *            lambda / (2 pi sigma xi_abs^2) *
 *            sum_{j : |p - q_j| <= (1 + eps) xi_abs} w_j cos(theta_j) G(r_j) P(r_j) / (1 + r_j^2)^2
 *   with r = |p - q| / xi_abs, cos(theta) = (p - q) . n / |p - q|,
 *   G(r) = exp(-(r - 1)^2 / (2 sigma^2)), exterior (pmc > 0): lambda = lambda1,
 *   P = (1 - i r)^2; interior: lambda = -lambda2, P = (1 + i r)^2
 *   (this is eq. 13 with the kernel of eq. 15 and zeta = xi + i eta).
 * q, nrm: n x 3 FP64 (positions, outward unit normals); w: n FP64 weights
 * (area elements; arc lengths in 2D) - FP64 in both precisions.  The
 * discrete decisions (nearest sample, membership, distance floor, and the
 * contact-ball test of samples within 1e-4 of its radius) are taken in FP64;
 * the kernel sum runs in the context's precision.  rho_out: complex,
 * g->n[0]*n[1]*n[2].  g, p: host structs.  Any grid shape is accepted.
 * The samples are put in Morton order in the context's workspace (about
 * 70 bytes per sample), which the next call of any entry point may reuse.
 * Errors: SDF_EINVAL (null pointer, n <= 0 or n > 2^30, bad grid, invalid
 * params), SDF_ENOMEM (workspace). */
int sdf_build(sdf_ctx ctx, const void *q, const void *nrm, const void *w, int64_t n,
              const sdf_grid *g, const sdf_params *p, void *rho_out, sdf_stream stream);

/* Alternative kernels of eq. 13.  The paper presents eq. 13 as a platform on
 * which scoring schemes differ only in the kernel phi, and compares its own
 * (eq. 15) with radial-basis and double-skin-layer affinities (Our Approach
 * section; Formulation section, the discussion before eq. 15 and Figure 8).
 * gb(x) below is g_sigma(x) = exp(-x^2 / (2 sigma^2)) / (sqrt(2 pi) sigma)
 * truncated to |x| <= eps (the truncated Gaussian the Formulation section
 * defines next to eq. 17t); R = radius > 0 is the probe radius of eq. 2 / 3a.
 *   SDF_PHI_SKELETAL        eq. 15 (sdf_build).
 *   SDF_PHI_INVERSE_SQUARE  phi = lambda(zeta) g_sigma(0) / (sqrt(2 pi) zeta^2):
 *                           eq. 15 with its medial Gaussian at its peak value, so
 *                           |phi| ~ |zeta|^-2 (Figure 8, middle) with the phase
 *                           -2 arg(zeta); membership, xi_floor and the
 *                           contact-region truncation as for the skeletal kernel.
 *   SDF_PHI_RADIAL          eq. 2 in its continuum form: skin and core are the
 *                           +R and -R offsets of the boundary, each point a
 *                           Gaussian shell of radius R:
 *                           rho(p) = sum_j w_j [lambda1 gb(|p - q_j - R n_j| / R - 1)
 *                                     + i lambda2 gb(|p - q_j + R n_j| / R - 1)];
 *                           xi_floor is not used.
 *   SDF_PHI_DSL             eq. 3a on the signed distance xi of the nearest
 *                           sample (as in sdf_build):
 *                           rho(p) = lambda1 gb(xi / R - 1) + i lambda2 gb(xi / R + 1);
 *                           defined on the boundary too, xi_floor is not used. */
typedef enum {
    SDF_PHI_SKELETAL = 0,
    SDF_PHI_INVERSE_SQUARE = 1,
    SDF_PHI_RADIAL = 2,
    SDF_PHI_DSL = 3
} sdf_phi_kind;
typedef struct {
    int32_t kind;   /* an sdf_phi_kind */
    double radius;  /* probe radius R (> 0) of SDF_PHI_RADIAL and SDF_PHI_DSL; ignored otherwise */
} sdf_phi;

/* sdf_build with the kernel `phi` (host struct; NULL = SDF_PHI_SKELETAL).
 * Same arguments, layout and decisions (FP64 nearest sample, membership and
 * truncation edges) as sdf_build.  The radial kernel sums over the 2 n offset
 * points within R (1 + eps) of a node (about 140 bytes of workspace per
 * sample); the DSL kernel needs only the nearest sample.
 * Errors: as sdf_build; SDF_EINVAL for an unknown kind, for the radial and
 * DSL kernels a radius that is not finite and > 0, and for the radial kernel
 * more than 2^29 samples. */
int sdf_build_phi(sdf_ctx ctx, const void *q, const void *nrm, const void *w, int64_t n,
                  const sdf_grid *g, const sdf_params *p, const sdf_phi *phi, void *rho_out, sdf_stream stream);

/* Adjoint of sdf_build with respect to its boundary samples (shape
 * gradients): for a complex cotangent field cot on the grid (context
 * precision, same layout as rho), the gradients of
 *   L = Re sum_p cot(p) rho(p)
 * with respect to the sample positions (grad_q, n x 3), normals (grad_n,
 * n x 3, unconstrained) and weights (grad_w, n), all FP64 device arrays that
 * the call overwrites.  The nearest sample, membership and contact ball of
 * every node are held (the SDF is piecewise smooth; these choices change only
 * on measure-zero sets).  With A = lambda / (2 pi sigma xi^2), u_j the unit
 * vector from q_j to the node, c_j = u_j . n_j, r_j = |p - q_j| / xi and
 * K = G P / (1 + r^2)^2:
 *   d rho / d w_j = A c_j K(r_j),   d rho / d n_j = A w_j K(r_j) u_j,
 *   d rho / d q_j = A w_j (-K (n_j - c_j u_j) / |p - q_j| - c_j K'(r_j) u_j / xi)
 * plus, for the nearest sample, -(d rho / d xi) u* with
 *   d rho / d xi = -(2 rho + A sum_j w_j c_j K'(r_j) r_j) / xi.
 * Computed in FP64 in both precisions; sums across node bricks use FP64
 * atomics, so the last bits may vary between runs.  Same inputs and
 * constraints as sdf_build; the samples' Morton order lives in the context's
 * workspace.
 * Errors: as sdf_build. */
int sdf_build_adjoint(sdf_ctx ctx, const void *q, const void *nrm, const void *w, int64_t n,
                      const sdf_grid *g, const sdf_params *p, const void *cot, double *grad_q,
                      double *grad_n, double *grad_w, sdf_stream stream);

/* Spectrum of the fixed part for the correlation (eq. 8):
 * spec_out(k) = N^-3 * sum_p rho_fixed(p) exp(-2 pi i k.p / N)  (N^-2 in 2D),
 * complex, same layout as the grid.  The grid must be N^3 or N^2 x 1 with N
 * in {8, 16, 32, 64, 96, 128}.  rho_fixed and spec_out may not alias.
 * Errors: SDF_EINVAL, SDF_EUNSUPPORTED. */
int sdf_spectrum(sdf_ctx ctx, const void *rho_fixed, const sdf_grid *g, void *spec_out, sdf_stream stream);

/* ------------------------------------------------------------ the search */

/* Score every integer translation of every rotation and reduce each rotation
 * to its peak (the search of the Formulation section; per-rotation FFT
 * correlation of the Implementation section).
 *   spec_fixed: output of sdf_spectrum for g_fixed.
 *   rho_moving: complex N_M^3 (or N_M^2 x 1) SDF of the moving part on its body
 *               box; w_moving: real, same size, per-node volume weights (h^3,
 *               h^2 in 2D, for the plain quadrature of eq. 8).
 *   quats (host): n_rot x 4 FP64 quaternions (non-zero, finite).
 * Outputs per rotation r (device):
 *   peak_score[r]   real, s = max_t Re f(R, t)
 *   peak_t[3r..]    int32 (tx, ty, tz) of the lowest flat index attaining s
 *   peak_nbhd[27r..] real, Re f at t* + (dx, dy, dz), offsets in {-1, 0, 1},
 *                   dz slowest, dx fastest, periodic (may be NULL)
 *   refined_t[3r..] FP64, t* + per-axis parabola vertex offset clamped to
 *                   [-1/2, 1/2], 0 where the curvature is not negative (may be NULL)
 * Constraints: h equal for both grids; the rotated body box plus its
 * stencil fits the periodic grid: ceil(sqrt(3) N_M) + 4 <= N in 3D,
 * ceil(sqrt(2) N_M) + 4 <= N in 2D.
 * Errors: SDF_EINVAL, SDF_EUNSUPPORTED, SDF_EHIP, SDF_ENOMEM. */
int score_rotations(sdf_ctx ctx, const void *spec_fixed, const sdf_grid *g_fixed,
                    const void *rho_moving, const void *w_moving, const sdf_grid *g_moving,
                    const double *quats, int64_t n_rot,
                    void *peak_score, int32_t *peak_t, void *peak_nbhd, double *refined_t,
                    sdf_stream stream);

/* Many pairs in one call (the uneven batch): each job is one pair with its
 * own spectrum, moving SDF, weights, quaternions (host) and outputs, as in
 * score_rotations.  Jobs may differ in N (8..128) and N_M.  FP32 contexts
 * group the jobs by grid size and run every group's rotations through one
 * persistent launch sequence per batch, reading per-pair descriptors; FP64
 * contexts (and "path" = 1) score the pairs one after the other.
 * Errors: as score_rotations, with the failing job's index in the message. */
typedef struct {
    const void *spec_fixed;
    sdf_grid g_fixed;
    const void *rho_moving;
    const void *w_moving;
    sdf_grid g_moving;
    const double *quats; /* host, n_rot x 4 */
    int64_t n_rot;
    void *peak_score;
    int32_t *peak_t;
    void *peak_nbhd;     /* may be NULL */
    double *refined_t;   /* may be NULL */
} sdf_pair_job;
int score_pairs(sdf_ctx ctx, const sdf_pair_job *jobs, int64_t n_jobs, sdf_stream stream);

/* Autotuner for the fused FP32 search of one grid-size class (N, planar,
 * N_M): times every candidate plan (rotations per batch in {32, 64, 128, 256},
 * rotations per pencil block in {2, 4}, three FFT radix schedules for the
 * sizes that use them; N = 64 and 128 use fixed two-pass transforms) on
 * synthetic inputs, rejects candidates whose peaks differ from the plain
 * multi-pass path by more than 1e-4 of the largest score on a probe set, and
 * keeps the fastest for this context (option "autotune" = 1 runs this on the
 * first search of each class).  report (host, may be NULL) receives a JSON
 * summary of all candidates, truncated to report_len - 1 bytes.  The
 * synthetic inputs are allocated for the duration of the call.
 * Errors: SDF_EINVAL, SDF_EUNSUPPORTED (FP64 context), SDF_ENOMEM, SDF_EHIP. */
int sdf_autotune(sdf_ctx ctx, const sdf_grid *g_fixed, const sdf_grid *g_moving, char *report, size_t report_len,
                 sdf_stream stream);

/* Full score volumes Re f(R, t) for every t of each rotation: vol_out is
 * real, n_rot x (grid size), same layout as the grid.  Same inputs and
 * constraints as score_rotations. */
int score_volume(sdf_ctx ctx, const void *spec_fixed, const sdf_grid *g_fixed,
                 const void *rho_moving, const void *w_moving, const sdf_grid *g_moving,
                 const double *quats, int64_t n_rot, void *vol_out, sdf_stream stream);

/* Reference search without the spreading window (eq. 8 by covariance,
 * rho(p, tau S) = rho(tau^-1 p, S)).  For each rotation R the moving part's
 * boundary samples are turned about its body-box centre c = o_M + h N_M / 2
 * (q -> c + R (q - c), n -> R n, in FP64; a planar box keeps c_z = o_M,z), its
 * SDF is built on the body-box nodes as sdf_build does, and the node values
 * times w_node sit on the fixed grid at the integer offsets k - N_M / 2, with
 * no window and no resampling:
 *   f(R, t) = sum_k w_node rho_R(x_k) rho_F((x_k / h + t) mod N),  score Re f.
 * The correlation, peak, 27-neighbourhood and sub-voxel refinement follow as
 * in score_rotations (same outputs and layouts).  q, nrm, w, n, p: the moving
 * part's boundary samples and SDF parameters as for sdf_build (device,
 * FP64).  N_M must be even.  O(N_M^3 n) per rotation: a reference that
 * measures what the B-spline window of score_rotations changes, not a fast
 * path.  The rotated samples, the box SDF and one correlation grid live in
 * the context's workspace.
 * Errors: SDF_EINVAL (null pointer, bad grids or params, odd N_M, n <= 0 or
 * n > 2^30, non-finite w_node), SDF_ENOMEM, SDF_EHIP. */
int score_rotations_direct(sdf_ctx ctx, const void *spec_fixed, const sdf_grid *g_fixed,
                           const void *q, const void *nrm, const void *w, int64_t n,
                           const sdf_grid *g_moving, const sdf_params *p, double w_node,
                           const double *quats, int64_t n_rot, void *peak_score, int32_t *peak_t,
                           void *peak_nbhd, double *refined_t, sdf_stream stream);

/* The rotated spread M_R on the fixed grid (complex, n_rot x grid size),
 * samples at +R x_k / h (not reflected).  Same constraints. */
int sdf_spread(sdf_ctx ctx, const sdf_grid *g_fixed, const void *rho_moving, const void *w_moving,
               const sdf_grid *g_moving, const double *quats, int64_t n_rot, void *grid_out,
               sdf_stream stream);

/* Unnormalised 3D (or 2D when nz = 1) DFT of a complex grid, out of place:
 * direction -1: out(k) = sum_p in(p) exp(-2 pi i k.p / N); +1: exp(+...).
 * Grid N^3 or N^2 x 1, N in {8, 16, 32, 64, 96, 128}. */
int sdf_fft(sdf_ctx ctx, const void *in, void *out, const sdf_grid *g, int direction, sdf_stream stream);

/* Top-k rotations by score: indices (int32, k) ordered by score descending,
 * ties by lower index.  scores: real, n.  1 <= k <= n. */
int sdf_topk(sdf_ctx ctx, const void *scores, int64_t n, int64_t k, int32_t *idx_out, sdf_stream stream);

/* ------------------------------------------------------------ refinement */

/* Pose value and gradients for gradient-based refinement (the validation
 * section's CG search over the score):
 *   f(t, q) = Re sum_k c_k Phi(R x_k / h + t),  Phi(y) = sum_p rho_F(p) B3(p - y),
 * which equals score_rotations' f(R, t) at integer t.
 *   rho_fixed: the fixed part's spatial SDF grid (not its spectrum).
 *   poses: B x 7 FP64 (t[3] in grid units, q[4] quaternion), device.
 *   score: real, B (required).
 *   grad_pose: FP64 B x 7 (df/dt, df/dq through R(q/|q|)), accumulated in FP64
 *              (may be NULL).
 *   grad_w: real N_M^3, sum over poses b of grad_scale[b] * Re(rho_M(x_k) Phi_b(y_k))
 *           (may be NULL).  grad_scale: FP64 B, device, NULL = all ones.
 * The B-spline stencil is recomputed, never stored.  Non-finite poses give
 * non-finite outputs for that pose.  Grid constraints as score_rotations
 * except that any N >= 4 works.
 * Errors: SDF_EINVAL, SDF_EHIP, SDF_ENOMEM. */
int score_grad(sdf_ctx ctx, const void *rho_fixed, const sdf_grid *g_fixed,
               const void *rho_moving, const void *w_moving, const sdf_grid *g_moving,
               const double *poses, int64_t B,
               void *score, double *grad_pose, void *grad_w, const double *grad_scale,
               sdf_stream stream);

/* Allocation-free score_grad, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight refinement or serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, semantics and outputs as
 * score_grad, but the kernels' scratch (the per-pose partial sums, and with
 * grad_w the per-pose-tile weight sums) lives in a fixed buffer of
 * SDF_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends (located once per device when a context is
 * created), never in the context's workspace; the call allocates nothing.
 * Limit: the problem must fit the buffer.  In FP32 with a 3D box of N_M^3
 * nodes it needs about 56 B x B x ceil(N_M / 8)^3, plus 4 B x N_M^3 per 16
 * poses with grad_w: 1 024 poses of a 64^3 box without grad_w fit, 256 poses
 * with it.  A larger problem fails with SDF_ENOMEM before anything is
 * enqueued.  Every call on one device shares that device's buffer, which
 * keeps the last call's contents: calls that overlap in time on one device
 * (other streams, threads or contexts) race and give wrong results.  Each
 * call writes all of the scratch it reads, so nothing needs clearing.
 * Errors: as score_grad; SDF_ENOMEM beyond the buffer; SDF_EHIP if the buffer
 * could not be located on the context's device. */
#define SDF_NOALLOC_SCRATCH_BYTES (32u << 20)
int score_grad_noalloc(sdf_ctx ctx, const void *rho_fixed, const sdf_grid *g_fixed,
                       const void *rho_moving, const void *w_moving, const sdf_grid *g_moving,
                       const double *poses, int64_t B,
                       void *score, double *grad_pose, void *grad_w, const double *grad_scale,
                       sdf_stream stream);

/* As score_grad, with the cotangent of the score with respect to the moving
 * part's coefficients c_k = w_k rho_M(x_k) (for gradients of rho_M itself,
 * and through sdf_build_adjoint, of the moving part's boundary samples):
 *   grad_c[k] = sum_b s_b Phi_b(R_b x_k / h + t_b)   (complex, N_M^3, context
 *   precision; s_b = grad_scale[b] or 1),
 * so that d(sum_b s_b f_b) = Re sum_k grad_c[k] dc_k.  The cotangent of
 * rho_M(x_k) is w_k grad_c[k]; grad_w (may be NULL) receives
 * Re(rho_M(x_k) grad_c[k]), as score_grad computes it.  grad_pose may be NULL.
 * Errors: as score_grad, and SDF_EINVAL for a NULL grad_c. */
int score_grad_coef(sdf_ctx ctx, const void *rho_fixed, const sdf_grid *g_fixed,
                    const void *rho_moving, const void *w_moving, const sdf_grid *g_moving,
                    const double *poses, int64_t B, void *score, double *grad_pose, void *grad_c,
                    void *grad_w, const double *grad_scale, sdf_stream stream);

/* Cotangent of sum_b s_b f_b with respect to the fixed part's field (the
 * adjoint of the gather in score_grad): every f_b is linear in rho_F, so
 *   grad_f(p) = sum_b s_b sum_k c_k B3(p - R_b x_k / h - t_b),   periodic,
 * with c_k = w_k rho_M(x_k) and s_b = grad_scale[b] (or 1): complex, the fixed
 * grid's size and layout, context precision, overwritten.  With
 * sdf_build_adjoint it gives the fixed part's shape gradients.  Sums use
 * atomic adds (the last bits may vary between runs).  Same constraints as
 * score_grad; rho_fixed is not needed.
 * Errors: SDF_EINVAL, SDF_ENOMEM, SDF_EHIP. */
int score_grad_fixed(sdf_ctx ctx, const sdf_grid *g_fixed, const void *rho_moving, const void *w_moving,
                     const sdf_grid *g_moving, const double *poses, int64_t B, const double *grad_scale,
                     void *grad_f, sdf_stream stream);

/* Backward pass of the pose scores for automatic differentiation (the
 * gradient-based refinement of the validation section): for an incoming
 * gradient g_b = grad_score[b] (FP64, device) of a loss L of the scores f_b,
 *   grad_pose[b]       = g_b d f_b / d pose_b          (FP64 B x 7, may be NULL)
 *   grad_w[k]          = sum_b g_b Re(rho_M(x_k) Phi_b(y_kb))   (real N_M^3, may be NULL)
 *   grad_rho_moving[k] = w_k sum_b g_b Phi_b(y_kb)     (complex N_M^3, may be NULL)
 *   grad_rho_fixed(p)  = sum_b g_b sum_k c_k B3(p - y_kb)   (complex fixed grid, may be NULL)
 * the last two being the cotangents of the fields, so that
 * dL = Re sum grad_rho . d rho (torch's complex gradient is their conjugate).
 * Each is what score_grad_coef / score_grad_fixed give, with the products
 * by g_b and w_k taken here.  Same inputs and constraints as score_grad;
 * rho_fixed may be NULL when only grad_rho_fixed is requested.  Outputs are
 * overwritten.
 * Errors: SDF_EINVAL (NULL input, no output requested), as score_grad. */
int score_grad_backward(sdf_ctx ctx, const void *rho_fixed, const sdf_grid *g_fixed,
                        const void *rho_moving, const void *w_moving, const sdf_grid *g_moving,
                        const double *poses, int64_t B, const double *grad_score,
                        double *grad_pose, void *grad_w, void *grad_rho_moving, void *grad_rho_fixed,
                        sdf_stream stream);

/* Chain rule for pose gradients kept from a forward score_grad call:
 * grad_pose_out[b][j] = grad_pose[b][j] * grad_score[b], FP64 B x 7, device
 * (grad_pose_out may equal grad_pose).
 * Errors: SDF_EINVAL. */
int score_grad_pose_chain(sdf_ctx ctx, const double *grad_pose, const double *grad_score, int64_t B,
                          double *grad_pose_out, sdf_stream stream);

/* ------------------------------------------------ nonequispaced route */

/* Octree-adaptive samples of the moving part (Implementation section: the
 * affinity varies most near the skeleton, so it is sampled on an octree,
 * deeper where it varies more, and the m' << m nonequispaced samples meet the
 * fixed part through a nonequispaced FFT).  The paper gives no subdivision
 * rule; this library's reading, on c_k = w_k rho_M(x_k) over the body box:
 *   - a cell is a cube of 2^l nodes per side (1 <= l <= max_level), aligned to
 *     multiples of 2^l; it is flat when over its nodes
 *       max Re c - min Re c < tau  and  max Im c - min Im c < tau,
 *       tau = tol * max_k max(|Re c_k|, |Im c_k|)
 *     (all in the context's precision; tol = 0 merges nothing);
 *   - each node goes to the highest flat cell above it, else stays a leaf of
 *     its own; a leaf is one sample at the cell centre, in grid units from
 *     the body origin (node k at k - N_M/2), carrying the sum of its nodes'
 *     coefficients (summed in FP64); leaves whose nodes are all zero are
 *     dropped;
 *   - order: 8^3 (planar 8^2) node blocks in flat x-fastest order, leaves in
 *     Morton order (x bit lowest) inside a block.
 * Arguments: rho_moving complex, w_moving real, N_M^3 or N_M^2 x 1 with N_M a
 * multiple of 8; max_level in [0, 3]; tol finite, >= 0.  Outputs (device,
 * capacity N_M^3 or N_M^2 leaves): pos_out real x 3 per leaf (z = 0 in 2D),
 * c_out complex, level_out int32 cell level l (may be NULL), count_out one
 * int64 = number of leaves.  Coefficients must be finite.
 * Errors: SDF_EINVAL, SDF_ENOMEM, SDF_EHIP. */
int octree_samples(sdf_ctx ctx, const void *rho_moving, const void *w_moving, const sdf_grid *g_moving,
                   double tol, int max_level, void *pos_out, void *c_out, int32_t *level_out,
                   int64_t *count_out, sdf_stream stream);

/* The search through the nonequispaced transform (Implementation section)
 * instead of the B-spline window: m samples at positions pos_k (real x 3,
 * grid units from the body origin, any values) with complex coefficients c_k
 * (from octree_samples, or every node of the body box) meet the fixed part
 * through its trigonometric interpolant,
 *   f(R, t) = sum_k c_k rho_F^trig(t + R pos_k),
 *   rho_F^trig(z) = N^-d sum_{kappa in [-N/2, N/2)^d} rho_F^(kappa) e^{2 pi i kappa.z / N},
 * evaluated per rotation by the type-1 transform of the reflected samples
 * -R pos_k: spreading with the "exponential of semicircle" kernel
 * exp(2.30 w (sqrt(1 - z^2) - 1)) over `width` nodes per axis of the 2x
 * oversampled grid, FFT, the N^d central modes divided by the kernel's
 * transform (Barnett, Magland and af Klinteberg, 2019; relative error about
 * 10^(1 - width)), product with spec_fixed, inverse FFT.  Peaks, 27-
 * neighbourhoods and sub-voxel offsets as in score_rotations.
 *   spec_fixed: output of sdf_spectrum; g_fixed N^3 or N^2 x 1 with N in
 *   {8, 16, 32, 64, 96, 128}; width in [2, 8]; 0 <= m <= 2^30 (m = 0 scores 0).
 *   quats (host): n_rot x 4 FP64.
 * Device workspace: up to 4 GiB per batch of rotations (the oversampled-grid
 * buffers, one N^d grid, the binned samples, 6 reals each, and for FP32 3D
 * peaks at N = 64 and 128 half a grid of folded spectra, per rotation of the
 * batch; about 60 rotations per batch at N = 128), at least one rotation's
 * worth.  FP32 3D peaks at N = 64 and 128 run the inverse transform and the
 * peak search through score_rotations' kernels (rotation pairs folded into
 * one complex transform); the other cases through the plain ones.
 * Errors: SDF_EINVAL, SDF_EUNSUPPORTED (N), SDF_ENOMEM, SDF_EHIP. */
int score_rotations_nfft(sdf_ctx ctx, const void *spec_fixed, const sdf_grid *g_fixed,
                         const void *pos, const void *c, int64_t m, int width,
                         const double *quats, int64_t n_rot,
                         void *peak_score, int32_t *peak_t, void *peak_nbhd, double *refined_t,
                         sdf_stream stream);

/* Full volumes Re f(R, t) of the nonequispaced route (real, n_rot x grid
 * size); same inputs and constraints as score_rotations_nfft. */
int score_volume_nfft(sdf_ctx ctx, const void *spec_fixed, const sdf_grid *g_fixed,
                      const void *pos, const void *c, int64_t m, int width,
                      const double *quats, int64_t n_rot, void *vol_out, sdf_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* SDFDOCK_H */
