// C ABI of the sdfdock library: argument validation, context and workspace
// management, and dispatch to the kernel launchers.  No exception escapes
// any entry point; every failure returns a code and records a message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <type_traits>
#include <string>
#include <vector>

#include "launch.hpp"
#include "sdfdock.h"

struct Tuned {
    int batch, group, radix;
};

struct GraphEntry {
    bool valid = false;
    std::vector<uintptr_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// Per-kernel timing with HIP events, enabled by the "profile" option.
struct Profiler : sdf::KernelTimer {
    struct Rec {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Rec> pending;
    std::map<std::string, std::pair<double, int64_t>> totals;
    bool ok = true;

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) ok = false;
        return e;
    }
    void events(const char* name, hipEvent_t* start, hipEvent_t* stop) override {
        Rec r{name, get(), get()};
        *start = r.a;
        *stop = r.b;
        pending.push_back(r);
    }
    void collect() {
        for (Rec& r : pending) {
            float ms = 0.f;
            if (r.a && r.b && hipEventSynchronize(r.b) == hipSuccess &&
                hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                auto& t = totals[r.name];
                t.first += ms;
                t.second += 1;
            }
            if (r.a) pool.push_back(r.a);
            if (r.b) pool.push_back(r.b);
        }
        pending.clear();
    }
    void release() {
        collect();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        pool.clear();
    }
};

struct sdf_ctx_s {
    int device = 0;
    sdf_dtype dtype = SDF_F32;
    size_t cap = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    std::string err;
    int64_t opt_path = 0;
    int64_t opt_batch = 64;
    int64_t opt_graph = 0;
    int64_t opt_pencil_group = 2;
    int64_t opt_profile = 0;
    int64_t opt_radix = 0;
    int64_t opt_autotune = 0;
    int64_t opt_autotune_reject = 0;  // candidates the autotuner must treat as failing its probe
    int num_cu = 256;
    std::map<uint64_t, Tuned> tuned;
    std::string last_report;
    // descriptors of the last fused search still resident in the workspace
    bool fused_cache_valid = false;
    void* fused_cache_base = nullptr;
    std::vector<char> fused_cache_jobs, fused_cache_rots;
    GraphEntry graph;
    Profiler prof;
    int64_t graph_captures = 0;
    int64_t graph_launches = 0;
    // "sdf_stats": sdf_build counts its node-sample pairs into stats_dev
    int64_t opt_sdf_stats = 0;
    unsigned long long* stats_dev = nullptr;
    // device address of this device's copy of `scratch` (score_grad_noalloc)
    void* scratch_ptr = nullptr;
    std::string scratch_err;
};

// Fixed scratch of the allocation-free entry point (score_grad_noalloc): the
// per-pose partial sums of the pose-gradient kernels.  Every device the
// library runs on holds its own copy until the process ends.  On the host
// this name is only a handle for hipGetSymbolAddress, never a device address.
constexpr size_t kScratchBytes = SDF_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

int fail(sdf_ctx ctx, int code, const std::string& msg) {
    g_err = msg;
    if (ctx) ctx->err = msg;
    return code;
}

int hip_fail(sdf_ctx ctx, hipError_t e, const char* where) {
    return fail(ctx, SDF_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define SDF_TRY_HIP(ctx, expr, where)                       \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Device address of `scratch` on `device`, looked up once per device (with
// that device current) and kept for the process; nullptr with a message in
// *err if the lookup fails.
void* scratch_address(int device, std::string* err) {
    static std::mutex mu;
    static std::map<int, void*> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it != addr.end()) return it->second;
    DeviceGuard dg(device);
    if (!dg.ok) {
        *err = "cannot select the device";
        return nullptr;
    }
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        *err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
        return nullptr;
    }
    addr[device] = p;
    return p;
}

bool finite(double v) { return std::isfinite(v); }

bool fft_size_ok(int n) { return n == 8 || n == 16 || n == 32 || n == 64 || n == 96 || n == 128; }

int check_grid(sdf_ctx ctx, const sdf_grid* g, const char* name) {
    if (!g) return fail(ctx, SDF_EINVAL, std::string(name) + " is NULL");
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] < 1) return fail(ctx, SDF_EINVAL, std::string(name) + ": node counts must be >= 1");
        if (!finite(g->origin[a])) return fail(ctx, SDF_EINVAL, std::string(name) + ": non-finite origin");
    }
    if (!(g->h > 0) || !finite(g->h)) return fail(ctx, SDF_EINVAL, std::string(name) + ": spacing must be > 0");
    const int64_t total = int64_t(g->n[0]) * g->n[1] * g->n[2];
    if (total > (int64_t(1) << 31)) return fail(ctx, SDF_EINVAL, std::string(name) + ": grid too large");
    return SDF_OK;
}

// fixed grid for correlation: N^3 or N^2 x 1, N a supported FFT size
int check_corr_grid(sdf_ctx ctx, const sdf_grid* g, const char* name) {
    int rc = check_grid(ctx, g, name);
    if (rc) return rc;
    if (g->n[0] != g->n[1] || (g->n[2] != g->n[0] && g->n[2] != 1))
        return fail(ctx, SDF_EINVAL, std::string(name) + ": must be N x N x N or N x N x 1");
    if (!fft_size_ok(g->n[0]))
        return fail(ctx, SDF_EUNSUPPORTED, std::string(name) + ": N must be one of 8, 16, 32, 64, 96, 128");
    return SDF_OK;
}

int check_pair(sdf_ctx ctx, const sdf_grid* gf, const sdf_grid* gm, bool need_fft) {
    int rc = need_fft ? check_corr_grid(ctx, gf, "g_fixed") : check_grid(ctx, gf, "g_fixed");
    if (rc) return rc;
    rc = check_grid(ctx, gm, "g_moving");
    if (rc) return rc;
    const bool planar = gf->n[2] == 1;
    if (!need_fft && (gf->n[0] != gf->n[1] || (gf->n[2] != gf->n[0] && !planar) || gf->n[0] < 4))
        return fail(ctx, SDF_EINVAL, "g_fixed: must be N x N x N or N x N x 1 with N >= 4");
    if (gm->n[0] != gm->n[1] || gm->n[2] != (planar ? 1 : gm->n[0]))
        return fail(ctx, SDF_EINVAL, "g_moving: must be N_M^3 (or N_M^2 x 1 with a planar fixed grid)");
    if (std::fabs(gf->h - gm->h) > 1e-12 * gf->h) return fail(ctx, SDF_EINVAL, "both grids must share h");
    const int N = gf->n[0], nm = gm->n[0];
    if (nm > N) return fail(ctx, SDF_EINVAL, "N_M > N");
    const double diag = std::sqrt(planar ? 2.0 : 3.0) * nm;
    // Every B-spline stencil index of the rotated body box then lies in
    // [-N/2, N/2) with a margin of at least 2.5e-3 cells for N_M <= 128, far
    // above FP32 position rounding; the fused slab layout relies on it.
    if (need_fft && (int(std::ceil(diag)) + 4 > N || diag > N - 4 - 1e-3))
        return fail(ctx, SDF_EINVAL, "rotated body box does not fit the periodic grid: need ceil(sqrt(d) N_M) + 4 <= N");
    return SDF_OK;
}

int check_params(sdf_ctx ctx, const sdf_params* p) {
    if (!p) return fail(ctx, SDF_EINVAL, "params is NULL");
    const double v[5] = {p->lambda1, p->lambda2, p->sigma, p->eps, p->xi_floor};
    for (double x : v)
        if (!finite(x)) return fail(ctx, SDF_EINVAL, "non-finite parameter");
    if (p->lambda1 <= 0 || p->lambda2 <= 0 || p->sigma <= 0 || p->eps < 0 || p->xi_floor < 0)
        return fail(ctx, SDF_EINVAL, "need lambda1, lambda2, sigma > 0 and eps, xi_floor >= 0");
    return SDF_OK;
}

int check_quats(sdf_ctx ctx, const double* q, int64_t n) {
    if (!q) return fail(ctx, SDF_EINVAL, "quats is NULL");
    if (n <= 0) return fail(ctx, SDF_EINVAL, "n_rot must be > 0");
    for (int64_t i = 0; i < n; ++i) {
        double s = 0;
        for (int a = 0; a < 4; ++a) {
            if (!finite(q[4 * i + a])) return fail(ctx, SDF_EINVAL, "non-finite quaternion");
            s += q[4 * i + a] * q[4 * i + a];
        }
        if (!(s > 0)) return fail(ctx, SDF_EINVAL, "zero quaternion");
    }
    return SDF_OK;
}

size_t esize(sdf_ctx ctx) { return ctx->dtype == SDF_F64 ? sizeof(double) : sizeof(float); }

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Carve {
    char* base;
    size_t off = 0;
    void* take(size_t bytes) {
        void* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    }
};

int ensure_ws(sdf_ctx ctx, size_t bytes) {
    if (bytes <= ctx->ws_bytes) return SDF_OK;
    if (ctx->cap && bytes > ctx->cap)
        return fail(ctx, SDF_ENOMEM, "workspace of " + std::to_string(bytes) + " bytes exceeds the cap of " +
                                         std::to_string(ctx->cap));
    if (ctx->ws) {
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, SDF_ENOMEM, std::string("workspace allocation failed: ") + hipGetErrorString(e));
    }
    ctx->ws = p;
    ctx->ws_bytes = bytes;
    return SDF_OK;
}

sdf::GridDesc desc(const sdf_grid* g) {
    return sdf::GridDesc{g->n[0], g->n[1], g->n[2], g->origin[0], g->origin[1], g->origin[2], g->h};
}

int64_t gsize(const sdf_grid* g) { return int64_t(g->n[0]) * g->n[1] * g->n[2]; }

void drop_graph(sdf_ctx ctx) {
    if (ctx->graph.exec) (void)hipGraphExecDestroy(ctx->graph.exec);
    if (ctx->graph.graph) (void)hipGraphDestroy(ctx->graph.graph);
    ctx->graph = GraphEntry{};
}

// ------------------------------------------------------------------ search core
// One pair of a search, as the ABI receives it.
struct PairIn {
    const void* spec;
    const sdf_grid* gf;
    const void* rho_m;
    const void* w_m;
    const sdf_grid* gm;
    const double* quats;
    int64_t n_rot;
    void* score;
    int32_t* t;
    void* nbhd;
    double* refined;
};

enum class Mode { Peaks, Volume };

// Plain path for one pair: one rotation per launch sequence.
template <typename T>
int plain_pair(sdf_ctx ctx, const PairIn& pr, Mode mode, void* vol_out, hipStream_t s) {
    ctx->fused_cache_valid = false;
    const int N = pr.gf->n[0];
    const bool planar = pr.gf->n[2] == 1;
    const int nm = pr.gm->n[0];
    const int64_t K = gsize(pr.gm), G = gsize(pr.gf);
    const int64_t n_rot = pr.n_rot;
    const int nparts = sdf::peak_parts<T>(N, planar);
    Carve cv{nullptr};
    cv.take(sizeof(double) * 4 * n_rot);
    cv.take(sizeof(double) * 9 * n_rot);
    cv.take(sizeof(T) * 9 * n_rot);
    cv.take(2 * sizeof(T) * K);
    cv.take(2 * sizeof(T) * G);
    cv.take(sizeof(T) * nparts);
    cv.take(sizeof(int) * nparts);
    int rc = ensure_ws(ctx, cv.off);
    if (rc) return rc;
    Carve c2{static_cast<char*>(ctx->ws)};
    double* qd = static_cast<double*>(c2.take(sizeof(double) * 4 * n_rot));
    double* r64 = static_cast<double*>(c2.take(sizeof(double) * 9 * n_rot));
    T* RT = static_cast<T*>(c2.take(sizeof(T) * 9 * n_rot));
    void* c = c2.take(2 * sizeof(T) * K);
    void* grid = c2.take(2 * sizeof(T) * G);
    T* pval = static_cast<T*>(c2.take(sizeof(T) * nparts));
    int* pidx = static_cast<int*>(c2.take(sizeof(int) * nparts));
    SDF_TRY_HIP(ctx, hipMemcpyAsync(qd, pr.quats, sizeof(double) * 4 * n_rot, hipMemcpyHostToDevice, s),
                "quaternion upload");
    SDF_TRY_HIP(ctx, sdf::launch_quat_to_rot<T>(qd, n_rot, r64, RT, s), "rotations");
    SDF_TRY_HIP(ctx, sdf::launch_coef<T>(pr.rho_m, static_cast<const T*>(pr.w_m), K, c, s), "coefficients");
    for (int64_t r = 0; r < n_rot; ++r) {
        SDF_TRY_HIP(ctx, sdf::launch_zero<T>(grid, G, s), "zero");
        SDF_TRY_HIP(ctx, sdf::launch_spread_atomic<T>(c, nm, planar, RT + 9 * r, 1, T(-1), N, grid, s), "spread");
        SDF_TRY_HIP(ctx, sdf::launch_fft3<T>(grid, N, planar, 1, -1, 1.0, s), "forward fft");
        SDF_TRY_HIP(ctx, sdf::launch_mul_spec<T>(grid, pr.spec, G, 1, s), "spectral product");
        SDF_TRY_HIP(ctx, sdf::launch_fft3<T>(grid, N, planar, 1, +1, 1.0, s), "inverse fft");
        if (mode == Mode::Volume) {
            SDF_TRY_HIP(ctx, sdf::launch_real_part<T>(grid, static_cast<T*>(vol_out) + r * G, G, s), "real part");
        } else {
            SDF_TRY_HIP(ctx,
                        sdf::launch_peak<T>(grid, true, N, planar, 1, pval, pidx, nparts,
                                            static_cast<T*>(pr.score) + r, pr.t + 3 * r,
                                            pr.nbhd ? static_cast<T*>(pr.nbhd) + 27 * r : nullptr,
                                            pr.refined ? pr.refined + 3 * r : nullptr, s),
                        "peak");
        }
    }
    return SDF_OK;
}

uint64_t class_key(int N, bool planar) { return uint64_t(N) * 2 + (planar ? 1 : 0); }

// Plan of one grid-size class: autotuned choice, else the context options.
sdf::FusedPlan plan_for(sdf_ctx ctx, int N, bool planar, int64_t rots_in_class) {
    sdf::FusedPlan fp{N, planar, int(ctx->opt_batch), int(ctx->opt_pencil_group), int(ctx->opt_radix),
                      ctx->num_cu};
    auto it = ctx->tuned.find(class_key(N, planar));
    if (it != ctx->tuned.end()) {
        fp.batch = it->second.batch;
        fp.pencil_group = it->second.group;
        fp.radix = it->second.radix;
    }
    if (fp.batch > rots_in_class) fp.batch = int((rots_in_class + 1) / 2 * 2);
    if (fp.batch < 2) fp.batch = 2;
    // the same number of launches, of equal size (no short tail launch)
    const int64_t launches = (rots_in_class + fp.batch - 1) / fp.batch;
    if (launches > 1) {
        const int64_t even = ((rots_in_class + launches - 1) / launches + 1) / 2 * 2;
        if (even < fp.batch) fp.batch = int(even);
    }
    return fp;
}

int autotune_class(sdf_ctx ctx, int N, bool planar, int n_m, hipStream_t s, std::string* report);

// Fused FP32 search over any number of pairs.  Pairs are grouped by grid
// size; each group's rotations run in batches through the persistent fused
// kernels, all reading per-pair descriptors.
int fused_pairs(sdf_ctx ctx, const std::vector<PairIn>& pairs, hipStream_t s) {
    const int nj = int(pairs.size());
    // classes in order of first appearance, jobs sorted by class
    std::vector<uint64_t> classes;
    for (const PairIn& p : pairs) {
        const uint64_t k = class_key(p.gf->n[0], p.gf->n[2] == 1);
        if (std::find(classes.begin(), classes.end(), k) == classes.end()) classes.push_back(k);
    }
    if (ctx->opt_autotune) {
        for (uint64_t k : classes) {
            if (ctx->tuned.count(k)) continue;
            int nm = 0;
            for (const PairIn& p : pairs)
                if (class_key(p.gf->n[0], p.gf->n[2] == 1) == k) nm = std::max(nm, p.gm->n[0]);
            int rc = autotune_class(ctx, int(k / 2), (k & 1) != 0, nm, s, nullptr);
            if (rc) return rc;
        }
    }
    std::vector<int> order;
    for (uint64_t k : classes)
        for (int j = 0; j < nj; ++j)
            if (class_key(pairs[j].gf->n[0], pairs[j].gf->n[2] == 1) == k) order.push_back(j);
    int64_t total_rot = 0;
    for (const PairIn& p : pairs) total_rot += p.n_rot;
    // workspace: descriptors, rotation inputs, per-pair coefficients and scales, prep scratch, batch buffers
    std::vector<sdf::FusedPlan> plans;
    std::vector<int64_t> class_rots(classes.size(), 0);
    for (size_t ci = 0; ci < classes.size(); ++ci)
        for (const PairIn& p : pairs)
            if (class_key(p.gf->n[0], p.gf->n[2] == 1) == classes[ci]) class_rots[ci] += p.n_rot;
    size_t batch_bytes = 0;
    for (size_t ci = 0; ci < classes.size(); ++ci) {
        plans.push_back(plan_for(ctx, int(classes[ci] / 2), (classes[ci] & 1) != 0, class_rots[ci]));
        batch_bytes = std::max(batch_bytes, sdf::fused_workspace_bytes(plans.back()));
    }
    auto grouped = [&](int j) { return sdf::fused_pair_grouped(pairs[j].gf->n[0], pairs[j].gf->n[2] == 1); };
    // one reordered spectrum copy per distinct spectrum (pairs may share the fixed part)
    std::vector<int> xsrc(nj, -1);
    for (int j = 0; j < nj; ++j) {
        if (!grouped(j)) continue;
        xsrc[j] = j;
        for (int i = 0; i < j; ++i)
            if (xsrc[i] == i && pairs[i].spec == pairs[j].spec && pairs[i].gf->n[0] == pairs[j].gf->n[0]) {
                xsrc[j] = i;
                break;
            }
    }
    auto carve = [&](char* base, std::vector<void*>* cptr, std::vector<float*>* sptr, std::vector<void*>* xptr,
                     sdf::FusedJob** jobs_d, sdf::FusedRot** rots_d, sdf::RotInput** rin_d, void** prep,
                     void** fused) {
        Carve cv{base};
        *jobs_d = static_cast<sdf::FusedJob*>(cv.take(sizeof(sdf::FusedJob) * nj));
        *rots_d = static_cast<sdf::FusedRot*>(cv.take(sizeof(sdf::FusedRot) * total_rot));
        *rin_d = static_cast<sdf::RotInput*>(cv.take(sizeof(sdf::RotInput) * total_rot));
        *prep = cv.take(sdf::fused_prep_scratch_bytes(nj));
        for (int j = 0; j < nj; ++j) {
            void* c = cv.take(sizeof(float) * 2 * size_t(gsize(pairs[j].gm)));
            float* sc = static_cast<float*>(cv.take(2 * sizeof(float)));
            void* x = xsrc[j] == j ? cv.take(sizeof(float) * 2 * size_t(gsize(pairs[j].gf))) : nullptr;
            if (cptr) (*cptr)[j] = c;
            if (sptr) (*sptr)[j] = sc;
            if (xptr) (*xptr)[j] = x;
        }
        if (xptr)
            for (int j = 0; j < nj; ++j)
                if (xsrc[j] >= 0 && xsrc[j] != j) (*xptr)[j] = (*xptr)[xsrc[j]];
        *fused = cv.take(batch_bytes);
        return cv.off;
    };
    sdf::FusedJob* jobs_d;
    sdf::FusedRot* rots_d;
    sdf::RotInput* rin_d;
    void *prep, *fused;
    const size_t need = carve(nullptr, nullptr, nullptr, nullptr, &jobs_d, &rots_d, &rin_d, &prep, &fused);
    int rc = ensure_ws(ctx, need);
    if (rc) return rc;
    std::vector<void*> cptr(nj), xptr(nj);
    std::vector<float*> sptr(nj);
    carve(static_cast<char*>(ctx->ws), &cptr, &sptr, &xptr, &jobs_d, &rots_d, &rin_d, &prep, &fused);
    // host tables (pinned staging is unnecessary: these are a few KB and copied synchronously)
    std::vector<sdf::FusedJob> jobs_h(nj);
    std::vector<sdf::RotInput> rin_h;
    rin_h.reserve(size_t(total_rot));
    for (int jj : order) {
        const PairIn& p = pairs[jj];
        jobs_h[jj] = sdf::FusedJob{cptr[jj], xptr[jj] ? xptr[jj] : p.spec, sptr[jj], static_cast<float*>(p.score), p.t,
                                   static_cast<float*>(p.nbhd), p.refined, p.gm->n[0], p.gf->n[2] == 1 ? 1 : 0};
        for (int64_t r = 0; r < p.n_rot; ++r) {
            sdf::RotInput ri;
            for (int a = 0; a < 4; ++a) ri.q[a] = p.quats[4 * r + a];
            ri.job = jj;
            ri.local = int(r);
            ri.n_m = p.gm->n[0];
            ri.N = p.gf->n[2] == 1 ? 0 : p.gf->n[0];
            rin_h.push_back(ri);
        }
    }
    // Upload the tables only when they differ from the ones still resident in
    // the workspace: a repeated search (same pairs, same rotations) enqueues
    // kernels only and never waits on the host.
    const char* jb = reinterpret_cast<const char*>(jobs_h.data());
    const char* rb = reinterpret_cast<const char*>(rin_h.data());
    const size_t jbytes = sizeof(sdf::FusedJob) * nj, rbytes = sizeof(sdf::RotInput) * total_rot;
    const bool cached = ctx->fused_cache_valid && ctx->fused_cache_base == ctx->ws &&
                        ctx->fused_cache_jobs.size() == jbytes && ctx->fused_cache_rots.size() == rbytes &&
                        std::memcmp(ctx->fused_cache_jobs.data(), jb, jbytes) == 0 &&
                        std::memcmp(ctx->fused_cache_rots.data(), rb, rbytes) == 0;
    if (!cached) {
        ctx->fused_cache_valid = false;
        SDF_TRY_HIP(ctx, hipMemcpyAsync(jobs_d, jb, jbytes, hipMemcpyHostToDevice, s), "job table upload");
        SDF_TRY_HIP(ctx, hipMemcpyAsync(rin_d, rb, rbytes, hipMemcpyHostToDevice, s), "rotation upload");
        // the copies read pageable host memory that goes out of scope on return
        SDF_TRY_HIP(ctx, hipStreamSynchronize(s), "upload");
        SDF_TRY_HIP(ctx, sdf::launch_rot_desc(rin_d, total_rot, rots_d, s), "rotations");
        ctx->fused_cache_jobs.assign(jb, jb + jbytes);
        ctx->fused_cache_rots.assign(rb, rb + rbytes);
        ctx->fused_cache_base = ctx->ws;
        ctx->fused_cache_valid = true;
    }
    for (int j = 0; j < nj; ++j)
        SDF_TRY_HIP(ctx,
                    sdf::launch_coef<float>(pairs[j].rho_m, static_cast<const float*>(pairs[j].w_m),
                                            gsize(pairs[j].gm), cptr[j], s),
                    "coefficients");
    for (int j = 0; j < nj; ++j)
        if (xsrc[j] == j)
            SDF_TRY_HIP(ctx, sdf::launch_spec_pair_group(pairs[j].spec, xptr[j], pairs[j].gf->n[0], s),
                        "spectrum column order");
    SDF_TRY_HIP(ctx, sdf::launch_fused_prep(jobs_d, nj, prep, s), "fixed-point scale");

    sdf::KernelTimer* kt = ctx->opt_profile ? &ctx->prof : nullptr;
    auto enqueue = [&]() -> hipError_t {
        int64_t r0 = 0;
        for (size_t ci = 0; ci < classes.size(); ++ci) {
            const sdf::FusedPlan& fp = plans[ci];
            for (int64_t b = 0; b < class_rots[ci]; b += fp.batch) {
                const int nb = int(std::min<int64_t>(fp.batch, class_rots[ci] - b));
                hipError_t e = sdf::launch_fused_batch(fp, rots_d + r0 + b, nb, jobs_d, fused, s, kt);
                if (e != hipSuccess) return e;
            }
            r0 += class_rots[ci];
        }
        return hipSuccess;
    };
    if (ctx->opt_graph && !kt && s != nullptr) {
        std::vector<uintptr_t> key = {uintptr_t(ctx->ws), uintptr_t(nj), uintptr_t(total_rot), uintptr_t(s)};
        for (const sdf::FusedPlan& fp : plans) {
            key.push_back(uintptr_t(fp.N) * 1315423911u + uintptr_t(fp.batch) * 31u + uintptr_t(fp.pencil_group) * 7u +
                          uintptr_t(fp.radix) + (fp.planar ? 977u : 0u));
        }
        for (int j = 0; j < nj; ++j) {
            const PairIn& p = pairs[j];
            key.insert(key.end(), {uintptr_t(p.spec), uintptr_t(p.score), uintptr_t(p.t), uintptr_t(p.nbhd),
                                   uintptr_t(p.refined), uintptr_t(p.n_rot), uintptr_t(p.gf->n[0]),
                                   uintptr_t(p.gf->n[2]), uintptr_t(p.gm->n[0])});
        }
        if (!(ctx->graph.valid && ctx->graph.key == key)) {
            drop_graph(ctx);
            SDF_TRY_HIP(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "graph capture begin");
            hipError_t e = enqueue();
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(s, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return hip_fail(ctx, e != hipSuccess ? e : e2, "graph capture");
            }
            hipGraphExec_t ex = nullptr;
            e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                return hip_fail(ctx, e, "graph instantiate");
            }
            ctx->graph.graph = g;
            ctx->graph.exec = ex;
            ctx->graph.key = key;
            ctx->graph.valid = true;
            ctx->graph_captures += 1;
        }
        SDF_TRY_HIP(ctx, hipGraphLaunch(ctx->graph.exec, s), "graph launch");
        ctx->graph_launches += 1;
        return SDF_OK;
    }
    SDF_TRY_HIP(ctx, enqueue(), "fused batch");
    return SDF_OK;
}

template <typename T>
int search_impl(sdf_ctx ctx, const std::vector<PairIn>& pairs, Mode mode, void* vol_out, hipStream_t s) {
    const bool fused = std::is_same<T, float>::value && mode == Mode::Peaks && ctx->opt_path != 1;
    if (fused) return fused_pairs(ctx, pairs, s);
    for (const PairIn& p : pairs) {
        int rc = plain_pair<T>(ctx, p, mode, vol_out, s);
        if (rc) return rc;
    }
    return SDF_OK;
}

// Autotuner: times candidate plans of one grid-size class on synthetic
// inputs and keeps the fastest whose peaks agree with the plain FP32 path.
int autotune_class(sdf_ctx ctx, int N, bool planar, int n_m, hipStream_t s, std::string* report) {
    if (ctx->dtype != SDF_F32) return SDF_OK;
    ctx->fused_cache_valid = false;
    const int nz = planar ? 1 : N;
    const int64_t G = int64_t(N) * N * nz;
    const int64_t K = int64_t(n_m) * n_m * (planar ? 1 : n_m);
    const int n_probe = 8;  // rotations compared with the plain path
    const int n_time = 256; // rotations timed per candidate (one launch at the largest batch)
    // synthetic pair in its own allocations (freed at the end)
    void *spec = nullptr, *rho = nullptr, *w = nullptr, *sc = nullptr, *tt = nullptr;
    void *sc_ref = nullptr, *tt_ref = nullptr;
    auto cleanup = [&]() {
        for (void* p : {spec, rho, w, sc, tt, sc_ref, tt_ref})
            if (p) (void)hipFree(p);
    };
    if (hipMalloc(&spec, 8 * G) != hipSuccess || hipMalloc(&rho, 8 * K) != hipSuccess ||
        hipMalloc(&w, 4 * K) != hipSuccess || hipMalloc(&sc, 4 * n_time) != hipSuccess ||
        hipMalloc(&tt, 12 * n_time) != hipSuccess || hipMalloc(&sc_ref, 4 * n_probe) != hipSuccess ||
        hipMalloc(&tt_ref, 12 * n_probe) != hipSuccess) {
        cleanup();
        (void)hipGetLastError();
        return fail(ctx, SDF_ENOMEM, "autotune allocation failed");
    }
    (void)sdf::launch_fill_random(spec, G, 11, 1e-3f, s);
    (void)sdf::launch_fill_random(rho, K, 12, 2.f, s);
    // w = 1: fill as complex pairs of (1, 1) over K/2 complex slots is awkward; use a real fill kernel
    {
        std::vector<float> ones(size_t(K), 1.f);  // unit body weights
        if (hipMemcpyAsync(w, ones.data(), 4 * K, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            cleanup();
            return fail(ctx, SDF_EHIP, "autotune upload failed");
        }
    }
    std::vector<double> q(4 * n_time);
    uint64_t st = 0x9e3779b97f4a7c15ull;
    auto rnd = [&]() {
        st ^= st << 13;
        st ^= st >> 7;
        st ^= st << 17;
        return double(st >> 11) * (1.0 / 9007199254740992.0);
    };
    for (int r = 0; r < n_time; ++r) {
        if (planar) {
            const double th = 2 * 3.14159265358979323846 * rnd();
            q[4 * r] = std::cos(th / 2);
            q[4 * r + 1] = 0;
            q[4 * r + 2] = 0;
            q[4 * r + 3] = std::sin(th / 2);
        } else {
            const double u1 = rnd(), u2 = rnd(), u3 = rnd();
            q[4 * r] = std::sqrt(u1) * std::cos(2 * 3.14159265358979323846 * u3);
            q[4 * r + 1] = std::sqrt(1 - u1) * std::sin(2 * 3.14159265358979323846 * u2);
            q[4 * r + 2] = std::sqrt(1 - u1) * std::cos(2 * 3.14159265358979323846 * u2);
            q[4 * r + 3] = std::sqrt(u1) * std::sin(2 * 3.14159265358979323846 * u3);
        }
    }
    sdf_grid gf{{N, N, nz}, {0, 0, 0}, 1.0};
    sdf_grid gm{{n_m, n_m, planar ? 1 : n_m}, {0, 0, 0}, 1.0};
    // reference peaks from the plain path
    PairIn ref{spec, &gf, rho, w, &gm, q.data(), n_probe, sc_ref, static_cast<int32_t*>(tt_ref), nullptr, nullptr};
    int rc = plain_pair<float>(ctx, ref, Mode::Peaks, nullptr, s);
    if (rc) {
        cleanup();
        return rc;
    }
    std::vector<float> s_ref(n_probe), s_got(n_probe);
    std::vector<int32_t> t_ref(3 * n_probe), t_got(3 * n_probe);
    if (hipStreamSynchronize(s) != hipSuccess || hipMemcpy(s_ref.data(), sc_ref, 4 * n_probe, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(t_ref.data(), tt_ref, 12 * n_probe, hipMemcpyDeviceToHost) != hipSuccess) {
        cleanup();
        return fail(ctx, SDF_EHIP, "autotune readback failed");
    }
    float smax = 0.f;
    for (float v : s_ref) smax = std::max(smax, std::fabs(v));
    const int64_t save_batch = ctx->opt_batch, save_group = ctx->opt_pencil_group, save_radix = ctx->opt_radix;
    const int64_t save_graph = ctx->opt_graph, save_auto = ctx->opt_autotune, save_prof = ctx->opt_profile;
    ctx->opt_graph = 0;
    ctx->opt_autotune = 0;
    ctx->opt_profile = 0;
    ctx->tuned.erase(class_key(N, planar));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    Tuned best{int(save_batch), int(save_group), int(save_radix)};
    float best_ms = 1e30f;
    std::string rep = "{\"N\": " + std::to_string(N) + ", \"n_m\": " + std::to_string(n_m) +
                      ", \"planar\": " + (planar ? "true" : "false") + ", \"candidates\": [";
    bool first = true;
    int cand = 0;
    for (int batch : {32, 64, 128, 256}) {
        for (int group : {2, 4}) {
            // N = 64 and 128 use fixed two-pass transforms: the schedule does not apply
            const int n_radix = (N == 64 || N == 128) ? 1 : 3;
            for (int radix = 0; radix < n_radix; ++radix) {
                ctx->opt_batch = batch;
                ctx->opt_pencil_group = group;
                ctx->opt_radix = radix;
                PairIn pr{spec, &gf, rho, w, &gm, q.data(), n_time, sc, static_cast<int32_t*>(tt), nullptr, nullptr};
                std::vector<PairIn> one{pr};
                rc = fused_pairs(ctx, one, s);  // warm-up and parity probe
                bool ok = rc == SDF_OK;
                if (ok) {
                    ok = hipStreamSynchronize(s) == hipSuccess &&
                         hipMemcpy(s_got.data(), sc, 4 * n_probe, hipMemcpyDeviceToHost) == hipSuccess &&
                         hipMemcpy(t_got.data(), tt, 12 * n_probe, hipMemcpyDeviceToHost) == hipSuccess;
                    for (int r = 0; ok && r < n_probe; ++r)
                        ok = std::fabs(s_got[r] - s_ref[r]) <= 1e-4f * smax + 1e-30f;
                }
                if ((ctx->opt_autotune_reject >> cand) & 1) ok = false;
                ++cand;
                float ms = -1.f;
                if (ok) {
                    (void)hipEventRecord(e0, s);
                    for (int it = 0; it < 2 && rc == SDF_OK; ++it) rc = fused_pairs(ctx, one, s);
                    (void)hipEventRecord(e1, s);
                    (void)hipEventSynchronize(e1);
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    ms /= 2;
                    if (rc == SDF_OK && ms < best_ms) {
                        best_ms = ms;
                        best = Tuned{batch, group, radix};
                    }
                }
                if (!first) rep += ", ";
                first = false;
                rep += "{\"batch\": " + std::to_string(batch) + ", \"group\": " + std::to_string(group) +
                       ", \"radix\": " + std::to_string(radix) + ", \"parity\": " + (ok ? "true" : "false") +
                       ", \"ms_per_rotation\": " + std::to_string(ms / n_time) + "}";
                rc = SDF_OK;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->opt_batch = save_batch;
    ctx->opt_pencil_group = save_group;
    ctx->opt_radix = save_radix;
    ctx->opt_graph = save_graph;
    ctx->opt_autotune = save_auto;
    ctx->opt_profile = save_prof;
    (void)hipStreamSynchronize(s);
    cleanup();
    if (best_ms >= 1e30f) return fail(ctx, SDF_EHIP, "autotune: no candidate passed the parity probe");
    ctx->tuned[class_key(N, planar)] = best;
    rep += "], \"chosen\": {\"batch\": " + std::to_string(best.batch) + ", \"group\": " +
           std::to_string(best.group) + ", \"radix\": " + std::to_string(best.radix) +
           ", \"ms_per_rotation\": " + std::to_string(best_ms / n_time) + "}}";
    if (report) *report = rep;
    ctx->last_report = rep;
    return SDF_OK;
}

}  // namespace

// =====================================================================  ABI

// Direct reference path: per rotation, SDF of the turned boundary samples on
// the body box, placed on the fixed grid without a window, then the plain
// path's transform, product, inverse and peak.
template <typename T>
int direct_impl(sdf_ctx ctx, const void* spec, const sdf_grid* gf, const double* q, const double* nrm,
                const double* w, int64_t ns, const sdf_grid* gm, const sdf_params* p, double w_node,
                const double* quats, int64_t n_rot, void* score, int32_t* t, void* nbhd, double* refined,
                hipStream_t s) {
    ctx->fused_cache_valid = false;
    const int N = gf->n[0];
    const bool planar = gf->n[2] == 1;
    const int nm = gm->n[0];
    const int64_t K = gsize(gm), G = gsize(gf);
    const int nparts = sdf::peak_parts<T>(N, planar);
    const size_t sdf_ws = sdf::sdf_build_workspace_bytes(ns);
    Carve cv{nullptr};
    cv.take(sizeof(double) * 4 * n_rot);
    cv.take(sizeof(double) * 9 * n_rot);
    cv.take(sizeof(T) * 9 * n_rot);
    cv.take(sizeof(double) * 3 * ns);
    cv.take(sizeof(double) * 3 * ns);
    cv.take(2 * sizeof(T) * K);
    cv.take(2 * sizeof(T) * G);
    cv.take(sizeof(T) * nparts);
    cv.take(sizeof(int) * nparts);
    cv.take(sdf_ws);
    int rc = ensure_ws(ctx, cv.off);
    if (rc) return rc;
    Carve c2{static_cast<char*>(ctx->ws)};
    double* qd = static_cast<double*>(c2.take(sizeof(double) * 4 * n_rot));
    double* r64 = static_cast<double*>(c2.take(sizeof(double) * 9 * n_rot));
    T* RT = static_cast<T*>(c2.take(sizeof(T) * 9 * n_rot));
    double* qr = static_cast<double*>(c2.take(sizeof(double) * 3 * ns));
    double* nr = static_cast<double*>(c2.take(sizeof(double) * 3 * ns));
    void* rho = c2.take(2 * sizeof(T) * K);
    void* grid = c2.take(2 * sizeof(T) * G);
    T* pval = static_cast<T*>(c2.take(sizeof(T) * nparts));
    int* pidx = static_cast<int*>(c2.take(sizeof(int) * nparts));
    void* wsb = c2.take(sdf_ws);
    const double c[3] = {gm->origin[0] + 0.5 * gm->h * nm, gm->origin[1] + 0.5 * gm->h * nm,
                         planar ? gm->origin[2] : gm->origin[2] + 0.5 * gm->h * nm};
    const sdf::ParamDesc pd{p->lambda1, p->lambda2, p->sigma, p->eps, p->xi_floor};
    SDF_TRY_HIP(ctx, hipMemcpyAsync(qd, quats, sizeof(double) * 4 * n_rot, hipMemcpyHostToDevice, s),
                "quaternion upload");
    SDF_TRY_HIP(ctx, sdf::launch_quat_to_rot<T>(qd, n_rot, r64, RT, s), "rotations");
    for (int64_t r = 0; r < n_rot; ++r) {
        SDF_TRY_HIP(ctx, sdf::launch_rotate_samples(q, nrm, ns, r64 + 9 * r, c, qr, nr, s), "rotate samples");
        SDF_TRY_HIP(ctx, sdf::launch_sdf_build<T>(qr, nr, w, ns, desc(gm), pd, sdf::kPhiSkeletal, rho, wsb, s),
                    "box sdf");
        SDF_TRY_HIP(ctx, sdf::launch_zero<T>(grid, G, s), "zero");
        SDF_TRY_HIP(ctx, sdf::launch_place_direct<T>(rho, nm, planar, T(w_node), N, grid, s), "place");
        SDF_TRY_HIP(ctx, sdf::launch_fft3<T>(grid, N, planar, 1, -1, 1.0, s), "forward fft");
        SDF_TRY_HIP(ctx, sdf::launch_mul_spec<T>(grid, spec, G, 1, s), "spectral product");
        SDF_TRY_HIP(ctx, sdf::launch_fft3<T>(grid, N, planar, 1, +1, 1.0, s), "inverse fft");
        SDF_TRY_HIP(ctx,
                    sdf::launch_peak<T>(grid, true, N, planar, 1, pval, pidx, nparts, static_cast<T*>(score) + r,
                                        t + 3 * r, nbhd ? static_cast<T*>(nbhd) + 27 * r : nullptr,
                                        refined ? refined + 3 * r : nullptr, s),
                    "peak");
    }
    return SDF_OK;
}

// Nonequispaced route: batches of rotations through the type-1 transform of
// the given samples, then the plain path's inverse FFT and peak (or real part).
constexpr size_t kNfftBudget = size_t(4096) << 20;  // per-batch workspace of the route

template <typename T>
int nfft_impl(sdf_ctx ctx, const void* spec, const sdf_grid* gf, const void* pos, const void* c, int64_t m, int w,
              const double* quats, int64_t n_rot, Mode mode, void* score, int32_t* t, void* nbhd, double* refined,
              void* vol_out, hipStream_t s) {
    ctx->fused_cache_valid = false;
    const int N = gf->n[0];
    const bool planar = gf->n[2] == 1;
    const int64_t G = gsize(gf);
    const size_t fine_bytes = sdf::nfft_grid_bytes(N, planar, sizeof(T));
    // rotations per batch: the per-rotation grids, x-pruned buffer and binned
    // samples within the budget
    // FP32 3D peaks at N = 64 and 128 go through the search path's inverse
    // kernels (rotation pairs folded into one inverse transform)
    const bool fused_peaks = std::is_same<T, float>::value && mode == Mode::Peaks && sdf::modes_peaks_supported(N, planar);
    const size_t per_rot = fine_bytes + 2 * sizeof(T) * size_t(G) + sdf::nfft_workspace_bytes(m, 1, N, planar, sizeof(T)) +
                           (fused_peaks ? sdf::modes_peaks_workspace_bytes(N, 2) / 2 : 0);
    int64_t B = std::max<int64_t>(1, std::min<int64_t>(n_rot, int64_t(kNfftBudget / per_rot)));
    if (m > 0) B = std::max<int64_t>(1, std::min<int64_t>(B, (int64_t(1) << 30) / m));  // binned samples < 2^31
    const int nparts = sdf::peak_parts<T>(N, planar);
    Carve cv{nullptr};
    cv.take(sizeof(double) * 4 * n_rot);
    cv.take(sizeof(double) * 9 * n_rot);
    cv.take(sizeof(T) * 9 * n_rot);
    cv.take(sizeof(T) * N);
    cv.take(fine_bytes * B);
    cv.take(2 * sizeof(T) * G * B);
    cv.take(sizeof(T) * nparts * B);
    cv.take(sizeof(int) * nparts * B);
    const size_t bin_bytes = sdf::nfft_workspace_bytes(m, int(B), N, planar, sizeof(T));
    cv.take(bin_bytes);
    const size_t peaks_bytes = fused_peaks ? sdf::modes_peaks_workspace_bytes(N, int(B)) : 0;
    cv.take(peaks_bytes);
    int rc = ensure_ws(ctx, cv.off);
    if (rc) return rc;
    Carve c2{static_cast<char*>(ctx->ws)};
    double* qd = static_cast<double*>(c2.take(sizeof(double) * 4 * n_rot));
    double* r64 = static_cast<double*>(c2.take(sizeof(double) * 9 * n_rot));
    T* RT = static_cast<T*>(c2.take(sizeof(T) * 9 * n_rot));
    T* inv = static_cast<T*>(c2.take(sizeof(T) * N));
    void* fine = c2.take(fine_bytes * B);
    void* grid = c2.take(2 * sizeof(T) * G * B);
    T* pval = static_cast<T*>(c2.take(sizeof(T) * nparts * B));
    int* pidx = static_cast<int*>(c2.take(sizeof(int) * nparts * B));
    void* bins = c2.take(bin_bytes);
    void* peaks_ws = c2.take(peaks_bytes);
    SDF_TRY_HIP(ctx, hipMemcpyAsync(qd, quats, sizeof(double) * 4 * n_rot, hipMemcpyHostToDevice, s),
                "quaternion upload");
    SDF_TRY_HIP(ctx, sdf::launch_quat_to_rot<T>(qd, n_rot, r64, RT, s), "rotations");
    SDF_TRY_HIP(ctx, sdf::launch_es_deconv<T>(N, w, inv, s), "deconvolution table");
    for (int64_t r0 = 0; r0 < n_rot; r0 += B) {
        const int nb = int(std::min<int64_t>(B, n_rot - r0));
        SDF_TRY_HIP(ctx,
                    sdf::launch_nfft_modes<T>(static_cast<const T*>(pos), c, m, RT + 9 * r0, nb, N, planar, w, inv,
                                              spec, fine, grid, bins, s, fused_peaks),
                    "nonequispaced transform");
        if (fused_peaks) {
            SDF_TRY_HIP(ctx,
                        sdf::launch_modes_peaks(N, grid, nb, 0, static_cast<float*>(score) + r0, t + 3 * r0,
                                                nbhd ? static_cast<float*>(nbhd) + 27 * r0 : nullptr,
                                                refined ? refined + 3 * r0 : nullptr, ctx->num_cu, peaks_ws, s),
                        "folded inverse and peaks");
            continue;
        }
        SDF_TRY_HIP(ctx, sdf::launch_fft3<T>(grid, N, planar, nb, +1, 1.0, s), "inverse fft");
        if (mode == Mode::Volume) {
            SDF_TRY_HIP(ctx, sdf::launch_real_part<T>(grid, static_cast<T*>(vol_out) + r0 * G, G * nb, s),
                        "real part");
        } else {
            SDF_TRY_HIP(ctx,
                        sdf::launch_peak<T>(grid, true, N, planar, nb, pval, pidx, nparts,
                                            static_cast<T*>(score) + r0, t + 3 * r0,
                                            nbhd ? static_cast<T*>(nbhd) + 27 * r0 : nullptr,
                                            refined ? refined + 3 * r0 : nullptr, s),
                        "peak");
        }
    }
    return SDF_OK;
}

int check_nfft_args(sdf_ctx ctx, const void* spec, const sdf_grid* gf, const void* pos, const void* c, int64_t m,
                    int w, const double* quats, int64_t n_rot) {
    if (!spec || (m > 0 && (!pos || !c))) return fail(ctx, SDF_EINVAL, "NULL array");
    int rc = check_grid(ctx, gf, "g_fixed");
    if (rc) return rc;
    const int N = gf->n[0];
    if (gf->n[1] != N || (gf->n[2] != N && gf->n[2] != 1))
        return fail(ctx, SDF_EINVAL, "g_fixed: must be N x N x N or N x N x 1");
    if (N != 8 && N != 16 && N != 32 && N != 64 && N != 96 && N != 128)
        return fail(ctx, SDF_EUNSUPPORTED, "g_fixed: the nonequispaced route needs N in {8, 16, 32, 64, 96, 128}");
    if (m < 0 || m > (int64_t(1) << 30)) return fail(ctx, SDF_EINVAL, "sample count must be in [0, 2^30]");
    if (w < 2 || w > 8) return fail(ctx, SDF_EINVAL, "kernel width must be in [2, 8]");
    rc = check_quats(ctx, quats, n_rot);
    if (rc) return rc;
    if (n_rot > (int64_t(1) << 24)) return fail(ctx, SDF_EINVAL, "n_rot too large");
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    return SDF_OK;
}

extern "C" {

int sdf_ctx_create(sdf_ctx* out, int device, sdf_dtype dtype, size_t workspace_cap_bytes) {
    if (!out) return fail(nullptr, SDF_EINVAL, "out is NULL");
    *out = nullptr;
    // a C caller may pass any int: read its bytes rather than the enum value,
    // which C++ does not define outside the enumerators' range
    int dt = 0;
    static_assert(sizeof(dtype) == sizeof(int), "sdf_dtype is int-sized");
    std::memcpy(&dt, &dtype, sizeof(int));
    if (dt != SDF_F32 && dt != SDF_F64) return fail(nullptr, SDF_EINVAL, "unknown dtype");
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return fail(nullptr, SDF_EHIP, "no such HIP device");
    }
    sdf_ctx ctx = new (std::nothrow) sdf_ctx_s();
    if (!ctx) return fail(nullptr, SDF_ENOMEM, "out of host memory");
    ctx->device = device;
    ctx->dtype = dtype;
    ctx->cap = workspace_cap_bytes;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->num_cu = prop.multiProcessorCount;
    ctx->scratch_ptr = scratch_address(device, &ctx->scratch_err);
    {
        DeviceGuard dg(device);
        if (dg.ok) sdf::fused_query_occupancy();
    }
    *out = ctx;
    return SDF_OK;
}

void sdf_ctx_destroy(sdf_ctx ctx) {
    if (!ctx) return;
    DeviceGuard dg(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->prof.release();
    drop_graph(ctx);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->stats_dev) (void)hipFree(ctx->stats_dev);
    delete ctx;
}

const char* sdf_last_error(sdf_ctx ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

int sdf_ctx_set_option(sdf_ctx ctx, const char* key, int64_t value) {
    if (!ctx || !key) return fail(ctx, SDF_EINVAL, "ctx or key is NULL");
    if (!std::strcmp(key, "path")) {
        if (value < 0 || value > 2) return fail(ctx, SDF_EINVAL, "path must be 0, 1 or 2");
        if (value == 2 && ctx->dtype != SDF_F32) return fail(ctx, SDF_EINVAL, "fused path is FP32 only");
        ctx->opt_path = value;
    } else if (!std::strcmp(key, "batch")) {
        if (value < 2 || value > 256 || (value & 1)) return fail(ctx, SDF_EINVAL, "batch must be even, 2..256");
        ctx->opt_batch = value;
        ctx->tuned.clear();
    } else if (!std::strcmp(key, "graph")) {
        if (value != 0 && value != 1) return fail(ctx, SDF_EINVAL, "graph must be 0 or 1");
        ctx->opt_graph = value;
    } else if (!std::strcmp(key, "pencil_group")) {
        if (value != 2 && value != 4) return fail(ctx, SDF_EINVAL, "pencil_group must be 2 or 4");
        ctx->opt_pencil_group = value;
    } else if (!std::strcmp(key, "profile")) {
        if (value != 0 && value != 1) return fail(ctx, SDF_EINVAL, "profile must be 0 or 1");
        ctx->opt_profile = value;
    } else if (!std::strcmp(key, "radix")) {
        if (value < 0 || value > 2) return fail(ctx, SDF_EINVAL, "radix must be 0, 1 or 2");
        ctx->opt_radix = value;
        ctx->tuned.clear();
    } else if (!std::strcmp(key, "autotune")) {
        if (value != 0 && value != 1) return fail(ctx, SDF_EINVAL, "autotune must be 0 or 1");
        ctx->opt_autotune = value;
    } else if (!std::strcmp(key, "autotune_reject")) {
        if (value < 0 || value >= (int64_t(1) << 24)) return fail(ctx, SDF_EINVAL, "autotune_reject: 24-bit mask");
        ctx->opt_autotune_reject = value;
    } else if (!std::strcmp(key, "sdf_stats")) {
        if (value != 0 && value != 1) return fail(ctx, SDF_EINVAL, "sdf_stats must be 0 or 1");
        ctx->opt_sdf_stats = value;
        if (ctx->stats_dev) {
            DeviceGuard dg(ctx->device);
            SDF_TRY_HIP(ctx, hipMemset(ctx->stats_dev, 0, 3 * sizeof(unsigned long long)), "statistics counters");
        }
    } else {
        return fail(ctx, SDF_EINVAL, std::string("unknown option ") + key);
    }
    return SDF_OK;
}

int sdf_ctx_get_option(sdf_ctx ctx, const char* key, int64_t* value) {
    if (!ctx || !key || !value) return fail(ctx, SDF_EINVAL, "NULL argument");
    if (!std::strcmp(key, "path")) *value = ctx->opt_path;
    else if (!std::strcmp(key, "batch")) *value = ctx->opt_batch;
    else if (!std::strcmp(key, "graph")) *value = ctx->opt_graph;
    else if (!std::strcmp(key, "pencil_group")) *value = ctx->opt_pencil_group;
    else if (!std::strcmp(key, "profile")) *value = ctx->opt_profile;
    else if (!std::strcmp(key, "radix")) *value = ctx->opt_radix;
    else if (!std::strcmp(key, "autotune")) *value = ctx->opt_autotune;
    else if (!std::strcmp(key, "num_cu")) *value = ctx->num_cu;
    else if (!std::strcmp(key, "graph_captures")) *value = ctx->graph_captures;
    else if (!std::strcmp(key, "graph_launches")) *value = ctx->graph_launches;
    else if (!std::strcmp(key, "sdf_stats")) *value = ctx->opt_sdf_stats;
    else if (!std::strcmp(key, "autotune_reject")) *value = ctx->opt_autotune_reject;
    else if (!std::strcmp(key, "sdf_pairs_nearest") || !std::strcmp(key, "sdf_pairs_sum") ||
             !std::strcmp(key, "sdf_pairs_in_ball")) {
        unsigned long long c[3] = {0, 0, 0};
        if (ctx->stats_dev) {
            DeviceGuard dg(ctx->device);
            SDF_TRY_HIP(ctx, hipMemcpy(c, ctx->stats_dev, sizeof(c), hipMemcpyDeviceToHost), "statistics counters");
        }
        *value = int64_t(c[key[10] == 'n' ? 0 : (key[10] == 's' ? 1 : 2)]);
    } else return fail(ctx, SDF_EINVAL, std::string("unknown option ") + key);
    return SDF_OK;
}

int sdf_ctx_stats(sdf_ctx ctx, const char* kernel, double* total_ms, int64_t* launches) {
    if (!ctx || !kernel || !total_ms || !launches) return fail(ctx, SDF_EINVAL, "NULL argument");
    DeviceGuard dg(ctx->device);
    ctx->prof.collect();
    auto it = ctx->prof.totals.find(kernel);
    *total_ms = it == ctx->prof.totals.end() ? 0.0 : it->second.first;
    *launches = it == ctx->prof.totals.end() ? 0 : it->second.second;
    return SDF_OK;
}

int sdf_ctx_stats_reset(sdf_ctx ctx) {
    if (!ctx) return fail(ctx, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    ctx->prof.collect();
    ctx->prof.totals.clear();
    return SDF_OK;
}

static int sdf_build_impl(sdf_ctx ctx, const void* q, const void* nrm, const void* w, int64_t n, const sdf_grid* g,
                          const sdf_params* p, const sdf_phi* phi, void* rho_out, sdf_stream stream) {
    if (!q || !nrm || !w || !rho_out) return fail(ctx, SDF_EINVAL, "NULL array");
    if (n <= 0) return fail(ctx, SDF_EINVAL, "sample count must be > 0");
    if (n > (int64_t(1) << 30)) return fail(ctx, SDF_EINVAL, "sample count must be <= 2^30");
    int rc = check_grid(ctx, g, "grid");
    if (rc) return rc;
    rc = check_params(ctx, p);
    if (rc) return rc;
    const int kind = phi ? phi->kind : SDF_PHI_SKELETAL;
    if (kind < SDF_PHI_SKELETAL || kind > SDF_PHI_DSL) return fail(ctx, SDF_EINVAL, "unknown phi kernel");
    const bool probe = kind == SDF_PHI_RADIAL || kind == SDF_PHI_DSL;
    if (probe && !(phi->radius > 0 && std::isfinite(phi->radius)))
        return fail(ctx, SDF_EINVAL, "the radial and DSL kernels need a finite probe radius > 0");
    if (kind == SDF_PHI_RADIAL && n > (int64_t(1) << 29))
        return fail(ctx, SDF_EINVAL, "the radial kernel takes at most 2^29 samples (2^30 offset points)");
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(ctx, SDF_EHIP, "cannot select device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    sdf::ParamDesc pd{p->lambda1, p->lambda2, p->sigma, p->eps, p->xi_floor};
    pd.radius = probe ? phi->radius : 0.0;
    const double* qd = static_cast<const double*>(q);
    const double* nd = static_cast<const double*>(nrm);
    const double* wd = static_cast<const double*>(w);
    ctx->fused_cache_valid = false;  // the Morton-ordered samples share the workspace
    rc = ensure_ws(ctx, sdf::sdf_build_workspace_bytes(n, kind));
    if (rc) return rc;
    unsigned long long* stats = nullptr;
    if (ctx->opt_sdf_stats && kind == SDF_PHI_SKELETAL) {
        if (!ctx->stats_dev) {
            SDF_TRY_HIP(ctx, hipMalloc(reinterpret_cast<void**>(&ctx->stats_dev), 3 * sizeof(unsigned long long)),
                        "statistics counters");
            SDF_TRY_HIP(ctx, hipMemsetAsync(ctx->stats_dev, 0, 3 * sizeof(unsigned long long), s),
                        "statistics counters");
        }
        stats = ctx->stats_dev;
    }
    hipError_t e = ctx->dtype == SDF_F64
                       ? sdf::launch_sdf_build<double>(qd, nd, wd, n, desc(g), pd, kind, rho_out, ctx->ws, s, stats)
                       : sdf::launch_sdf_build<float>(qd, nd, wd, n, desc(g), pd, kind, rho_out, ctx->ws, s, stats);
    if (e != hipSuccess) return hip_fail(ctx, e, "sdf_build");
    return SDF_OK;
}

int sdf_build(sdf_ctx ctx, const void* q, const void* nrm, const void* w, int64_t n, const sdf_grid* g,
              const sdf_params* p, void* rho_out, sdf_stream stream) {
    return sdf_build_impl(ctx, q, nrm, w, n, g, p, nullptr, rho_out, stream);
}

int sdf_build_phi(sdf_ctx ctx, const void* q, const void* nrm, const void* w, int64_t n, const sdf_grid* g,
                  const sdf_params* p, const sdf_phi* phi, void* rho_out, sdf_stream stream) {
    return sdf_build_impl(ctx, q, nrm, w, n, g, p, phi, rho_out, stream);
}

int sdf_build_adjoint(sdf_ctx ctx, const void* q, const void* nrm, const void* w, int64_t n, const sdf_grid* g,
                      const sdf_params* p, const void* cot, double* grad_q, double* grad_n, double* grad_w,
                      sdf_stream stream) {
    if (!q || !nrm || !w || !cot || !grad_q || !grad_n || !grad_w) return fail(ctx, SDF_EINVAL, "NULL array");
    if (n <= 0 || n > (int64_t(1) << 30)) return fail(ctx, SDF_EINVAL, "sample count must be in [1, 2^30]");
    int rc = check_grid(ctx, g, "grid");
    if (rc) return rc;
    rc = check_params(ctx, p);
    if (rc) return rc;
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(ctx, SDF_EHIP, "cannot select device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const sdf::ParamDesc pd{p->lambda1, p->lambda2, p->sigma, p->eps, p->xi_floor};
    const double* qd = static_cast<const double*>(q);
    const double* nd = static_cast<const double*>(nrm);
    const double* wd = static_cast<const double*>(w);
    ctx->fused_cache_valid = false;  // the Morton-ordered samples share the workspace
    rc = ensure_ws(ctx, sdf::sdf_build_workspace_bytes(n));
    if (rc) return rc;
    hipError_t e = ctx->dtype == SDF_F64
                       ? sdf::launch_sdf_adjoint<double>(qd, nd, wd, n, desc(g), pd, cot, grad_q, grad_n, grad_w,
                                                         ctx->ws, s)
                       : sdf::launch_sdf_adjoint<float>(qd, nd, wd, n, desc(g), pd, cot, grad_q, grad_n, grad_w,
                                                        ctx->ws, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "sdf_build_adjoint");
    return SDF_OK;
}

int sdf_fft(sdf_ctx ctx, const void* in, void* out, const sdf_grid* g, int direction, sdf_stream stream) {
    if (!in || !out) return fail(ctx, SDF_EINVAL, "NULL array");
    if (direction != -1 && direction != 1) return fail(ctx, SDF_EINVAL, "direction must be -1 or +1");
    int rc = check_corr_grid(ctx, g, "grid");
    if (rc) return rc;
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t bytes = 2 * esize(ctx) * size_t(gsize(g));
    if (in != out) SDF_TRY_HIP(ctx, hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, s), "copy");
    const bool planar = g->n[2] == 1;
    hipError_t e = ctx->dtype == SDF_F64 ? sdf::launch_fft3<double>(out, g->n[0], planar, 1, direction, 1.0, s)
                                         : sdf::launch_fft3<float>(out, g->n[0], planar, 1, direction, 1.0, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "fft");
    return SDF_OK;
}

int sdf_spectrum(sdf_ctx ctx, const void* rho_fixed, const sdf_grid* g, void* spec_out, sdf_stream stream) {
    if (!rho_fixed || !spec_out) return fail(ctx, SDF_EINVAL, "NULL array");
    if (rho_fixed == spec_out) return fail(ctx, SDF_EINVAL, "rho_fixed and spec_out alias");
    int rc = check_corr_grid(ctx, g, "grid");
    if (rc) return rc;
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t bytes = 2 * esize(ctx) * size_t(gsize(g));
    SDF_TRY_HIP(ctx, hipMemcpyAsync(spec_out, rho_fixed, bytes, hipMemcpyDeviceToDevice, s), "copy");
    const bool planar = g->n[2] == 1;
    const double scale = 1.0 / double(gsize(g));
    hipError_t e = ctx->dtype == SDF_F64 ? sdf::launch_fft3<double>(spec_out, g->n[0], planar, 1, -1, scale, s)
                                         : sdf::launch_fft3<float>(spec_out, g->n[0], planar, 1, -1, scale, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "spectrum fft");
    return SDF_OK;
}

int score_rotations(sdf_ctx ctx, const void* spec_fixed, const sdf_grid* g_fixed, const void* rho_moving,
                    const void* w_moving, const sdf_grid* g_moving, const double* quats, int64_t n_rot,
                    void* peak_score, int32_t* peak_t, void* peak_nbhd, double* refined_t, sdf_stream stream) {
    if (!spec_fixed || !rho_moving || !w_moving || !peak_score || !peak_t)
        return fail(ctx, SDF_EINVAL, "NULL array");
    int rc = check_pair(ctx, g_fixed, g_moving, true);
    if (rc) return rc;
    rc = check_quats(ctx, quats, n_rot);
    if (rc) return rc;
    if (n_rot > (int64_t(1) << 28)) return fail(ctx, SDF_EINVAL, "n_rot too large");
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<PairIn> pairs{PairIn{spec_fixed, g_fixed, rho_moving, w_moving, g_moving, quats, n_rot, peak_score,
                                     peak_t, peak_nbhd, refined_t}};
    if (ctx->dtype == SDF_F64) return search_impl<double>(ctx, pairs, Mode::Peaks, nullptr, s);
    return search_impl<float>(ctx, pairs, Mode::Peaks, nullptr, s);
}

int score_pairs(sdf_ctx ctx, const sdf_pair_job* jobs, int64_t n_jobs, sdf_stream stream) {
    if (!jobs || n_jobs <= 0) return fail(ctx, SDF_EINVAL, "need n_jobs > 0 and a job array");
    if (n_jobs > (int64_t(1) << 20)) return fail(ctx, SDF_EINVAL, "too many jobs");
    std::vector<PairIn> pairs;
    int64_t total = 0;
    for (int64_t j = 0; j < n_jobs; ++j) {
        const sdf_pair_job& jb = jobs[j];
        if (!jb.spec_fixed || !jb.rho_moving || !jb.w_moving || !jb.peak_score || !jb.peak_t)
            return fail(ctx, SDF_EINVAL, "job " + std::to_string(j) + ": NULL array");
        int rc = check_pair(ctx, &jb.g_fixed, &jb.g_moving, true);
        if (rc) return fail(ctx, rc, "job " + std::to_string(j) + ": " + g_err);
        rc = check_quats(ctx, jb.quats, jb.n_rot);
        if (rc) return fail(ctx, rc, "job " + std::to_string(j) + ": " + g_err);
        total += jb.n_rot;
        pairs.push_back(PairIn{jb.spec_fixed, &jb.g_fixed, jb.rho_moving, jb.w_moving, &jb.g_moving, jb.quats,
                               jb.n_rot, jb.peak_score, jb.peak_t, jb.peak_nbhd, jb.refined_t});
    }
    if (total > (int64_t(1) << 28)) return fail(ctx, SDF_EINVAL, "too many rotations");
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ctx->dtype == SDF_F64) return search_impl<double>(ctx, pairs, Mode::Peaks, nullptr, s);
    return search_impl<float>(ctx, pairs, Mode::Peaks, nullptr, s);
}

int sdf_autotune(sdf_ctx ctx, const sdf_grid* g_fixed, const sdf_grid* g_moving, char* report, size_t report_len,
                 sdf_stream stream) {
    int rc = check_pair(ctx, g_fixed, g_moving, true);
    if (rc) return rc;
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    if (ctx->dtype != SDF_F32) return fail(ctx, SDF_EUNSUPPORTED, "autotuning applies to FP32 contexts");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::string rep;
    rc = autotune_class(ctx, g_fixed->n[0], g_fixed->n[2] == 1, g_moving->n[0], s, &rep);
    if (rc) return rc;
    if (report && report_len > 0) {
        const size_t n = std::min(report_len - 1, rep.size());
        std::memcpy(report, rep.data(), n);
        report[n] = 0;
    }
    return SDF_OK;
}

int score_volume(sdf_ctx ctx, const void* spec_fixed, const sdf_grid* g_fixed, const void* rho_moving,
                 const void* w_moving, const sdf_grid* g_moving, const double* quats, int64_t n_rot, void* vol_out,
                 sdf_stream stream) {
    if (!spec_fixed || !rho_moving || !w_moving || !vol_out) return fail(ctx, SDF_EINVAL, "NULL array");
    int rc = check_pair(ctx, g_fixed, g_moving, true);
    if (rc) return rc;
    rc = check_quats(ctx, quats, n_rot);
    if (rc) return rc;
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<PairIn> pairs{PairIn{spec_fixed, g_fixed, rho_moving, w_moving, g_moving, quats, n_rot, nullptr,
                                     nullptr, nullptr, nullptr}};
    if (ctx->dtype == SDF_F64) return search_impl<double>(ctx, pairs, Mode::Volume, vol_out, s);
    return search_impl<float>(ctx, pairs, Mode::Volume, vol_out, s);
}

int score_rotations_direct(sdf_ctx ctx, const void* spec_fixed, const sdf_grid* g_fixed, const void* q,
                           const void* nrm, const void* w, int64_t n, const sdf_grid* g_moving, const sdf_params* p,
                           double w_node, const double* quats, int64_t n_rot, void* peak_score, int32_t* peak_t,
                           void* peak_nbhd, double* refined_t, sdf_stream stream) {
    if (!spec_fixed || !q || !nrm || !w || !peak_score || !peak_t) return fail(ctx, SDF_EINVAL, "NULL array");
    if (n <= 0 || n > (int64_t(1) << 30)) return fail(ctx, SDF_EINVAL, "sample count must be in [1, 2^30]");
    if (!std::isfinite(w_node)) return fail(ctx, SDF_EINVAL, "w_node must be finite");
    int rc = check_pair(ctx, g_fixed, g_moving, true);
    if (rc) return rc;
    if (g_moving->n[0] % 2) return fail(ctx, SDF_EINVAL, "the direct placement needs an even N_M");
    rc = check_params(ctx, p);
    if (rc) return rc;
    rc = check_quats(ctx, quats, n_rot);
    if (rc) return rc;
    if (n_rot > (int64_t(1) << 24)) return fail(ctx, SDF_EINVAL, "n_rot too large");
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double* qd = static_cast<const double*>(q);
    const double* nd = static_cast<const double*>(nrm);
    const double* wd = static_cast<const double*>(w);
    if (ctx->dtype == SDF_F64)
        return direct_impl<double>(ctx, spec_fixed, g_fixed, qd, nd, wd, n, g_moving, p, w_node, quats, n_rot,
                                   peak_score, peak_t, peak_nbhd, refined_t, s);
    return direct_impl<float>(ctx, spec_fixed, g_fixed, qd, nd, wd, n, g_moving, p, w_node, quats, n_rot, peak_score,
                              peak_t, peak_nbhd, refined_t, s);
}

int sdf_spread(sdf_ctx ctx, const sdf_grid* g_fixed, const void* rho_moving, const void* w_moving,
               const sdf_grid* g_moving, const double* quats, int64_t n_rot, void* grid_out, sdf_stream stream) {
    if (!rho_moving || !w_moving || !grid_out) return fail(ctx, SDF_EINVAL, "NULL array");
    int rc = check_pair(ctx, g_fixed, g_moving, true);
    if (rc) return rc;
    rc = check_quats(ctx, quats, n_rot);
    if (rc) return rc;
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    ctx->fused_cache_valid = false;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t K = gsize(g_moving), G = gsize(g_fixed);
    const bool planar = g_fixed->n[2] == 1;
    const size_t es = esize(ctx);
    Carve cv{nullptr};
    cv.take(sizeof(double) * 4 * n_rot);
    cv.take(sizeof(double) * 9 * n_rot);
    cv.take(es * 9 * n_rot);
    cv.take(2 * es * K);
    rc = ensure_ws(ctx, cv.off);
    if (rc) return rc;
    Carve c2{static_cast<char*>(ctx->ws)};
    double* qd = static_cast<double*>(c2.take(sizeof(double) * 4 * n_rot));
    double* r64 = static_cast<double*>(c2.take(sizeof(double) * 9 * n_rot));
    void* rT = c2.take(es * 9 * n_rot);
    void* c = c2.take(2 * es * K);
    SDF_TRY_HIP(ctx, hipMemcpyAsync(qd, quats, sizeof(double) * 4 * n_rot, hipMemcpyHostToDevice, s), "upload");
    hipError_t e;
    if (ctx->dtype == SDF_F64) {
        e = sdf::launch_quat_to_rot<double>(qd, n_rot, r64, static_cast<double*>(rT), s);
        if (e == hipSuccess) e = sdf::launch_coef<double>(rho_moving, static_cast<const double*>(w_moving), K, c, s);
        if (e == hipSuccess) e = sdf::launch_zero<double>(grid_out, G * n_rot, s);
        if (e == hipSuccess)
            e = sdf::launch_spread_atomic<double>(c, g_moving->n[0], planar, static_cast<double*>(rT), int(n_rot),
                                                  1.0, g_fixed->n[0], grid_out, s);
    } else {
        e = sdf::launch_quat_to_rot<float>(qd, n_rot, r64, static_cast<float*>(rT), s);
        if (e == hipSuccess) e = sdf::launch_coef<float>(rho_moving, static_cast<const float*>(w_moving), K, c, s);
        if (e == hipSuccess) e = sdf::launch_zero<float>(grid_out, G * n_rot, s);
        if (e == hipSuccess)
            e = sdf::launch_spread_atomic<float>(c, g_moving->n[0], planar, static_cast<float*>(rT), int(n_rot),
                                                 1.0f, g_fixed->n[0], grid_out, s);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "spread");
    return SDF_OK;
}

int sdf_topk(sdf_ctx ctx, const void* scores, int64_t n, int64_t k, int32_t* idx_out, sdf_stream stream) {
    if (!scores || !idx_out) return fail(ctx, SDF_EINVAL, "NULL array");
    if (n <= 0 || k < 1 || k > n) return fail(ctx, SDF_EINVAL, "need 1 <= k <= n");
    if (n > (int64_t(1) << 30)) return fail(ctx, SDF_EINVAL, "n too large");
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    ctx->fused_cache_valid = false;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = ensure_ws(ctx, sdf::topk_workspace_bytes(n));
    if (rc) return rc;
    hipError_t e = ctx->dtype == SDF_F64
                       ? sdf::launch_topk<double>(static_cast<const double*>(scores), n, k, ctx->ws, idx_out, s)
                       : sdf::launch_topk<float>(static_cast<const float*>(scores), n, k, ctx->ws, idx_out, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "topk");
    return SDF_OK;
}

// scratch == nullptr: the context's workspace (grown as needed); otherwise
// the fixed scratch buffer of score_grad_noalloc, which bounds the problem.
static int score_grad_impl(sdf_ctx ctx, const void* rho_fixed, const sdf_grid* g_fixed, const void* rho_moving,
                           const void* w_moving, const sdf_grid* g_moving, const double* poses, int64_t B,
                           void* score, double* grad_pose, void* grad_w, void* grad_c, const double* grad_scale,
                           sdf_stream stream, void* scratch_buf = nullptr) {
    if (!rho_fixed || !rho_moving || !w_moving || !poses || !score) return fail(ctx, SDF_EINVAL, "NULL array");
    if (B <= 0) return fail(ctx, SDF_EINVAL, "B must be > 0");
    if (B > (int64_t(1) << 24)) return fail(ctx, SDF_EINVAL, "B too large");
    int rc = check_pair(ctx, g_fixed, g_moving, false);
    if (rc) return rc;
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(ctx, SDF_EHIP, "cannot select device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool planar = g_fixed->n[2] == 1;
    const int N = g_fixed->n[0], nm = g_moving->n[0];
    const int wmode = grad_c ? 2 : (grad_w ? 1 : 0);
    size_t need = ctx->dtype == SDF_F64 ? sdf::grad_workspace_bytes<double>(B, N, nm, planar, wmode)
                                        : sdf::grad_workspace_bytes<float>(B, N, nm, planar, wmode);
    void* ws = scratch_buf;
    if (scratch_buf) {
        if (need > kScratchBytes)
            return fail(ctx, SDF_ENOMEM, "score_grad_noalloc needs " + std::to_string(need) +
                                             " bytes of scratch, more than its fixed " +
                                             std::to_string(kScratchBytes) + " (fewer poses per call, or no grad_w)");
    } else {
        ctx->fused_cache_valid = false;
        rc = ensure_ws(ctx, need);
        if (rc) return rc;
        ws = ctx->ws;
    }
    hipError_t e;
    if (ctx->dtype == SDF_F64)
        e = sdf::launch_score_grad<double>(rho_fixed, N, planar, rho_moving, static_cast<const double*>(w_moving), nm,
                                           poses, B, static_cast<double*>(score), grad_pose,
                                           static_cast<double*>(grad_w), static_cast<double*>(grad_c), grad_scale,
                                           ws, s);
    else
        e = sdf::launch_score_grad<float>(rho_fixed, N, planar, rho_moving, static_cast<const float*>(w_moving), nm,
                                          poses, B, static_cast<float*>(score), grad_pose,
                                          static_cast<float*>(grad_w), static_cast<float*>(grad_c), grad_scale,
                                          ws, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "score_grad");
    return SDF_OK;
}

int score_grad(sdf_ctx ctx, const void* rho_fixed, const sdf_grid* g_fixed, const void* rho_moving,
               const void* w_moving, const sdf_grid* g_moving, const double* poses, int64_t B, void* score,
               double* grad_pose, void* grad_w, const double* grad_scale, sdf_stream stream) {
    return score_grad_impl(ctx, rho_fixed, g_fixed, rho_moving, w_moving, g_moving, poses, B, score, grad_pose,
                           grad_w, nullptr, grad_scale, stream);
}

int score_grad_noalloc(sdf_ctx ctx, const void* rho_fixed, const sdf_grid* g_fixed, const void* rho_moving,
                       const void* w_moving, const sdf_grid* g_moving, const double* poses, int64_t B, void* score,
                       double* grad_pose, void* grad_w, const double* grad_scale, sdf_stream stream) {
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    if (!ctx->scratch_ptr)
        return fail(ctx, SDF_EHIP, "the scratch buffer of device " + std::to_string(ctx->device) +
                                       " was not located: " + ctx->scratch_err);
    return score_grad_impl(ctx, rho_fixed, g_fixed, rho_moving, w_moving, g_moving, poses, B, score, grad_pose,
                           grad_w, nullptr, grad_scale, stream, ctx->scratch_ptr);
}

int score_grad_coef(sdf_ctx ctx, const void* rho_fixed, const sdf_grid* g_fixed, const void* rho_moving,
                    const void* w_moving, const sdf_grid* g_moving, const double* poses, int64_t B, void* score,
                    double* grad_pose, void* grad_c, void* grad_w, const double* grad_scale, sdf_stream stream) {
    if (!grad_c) return fail(ctx, SDF_EINVAL, "grad_c is NULL");
    return score_grad_impl(ctx, rho_fixed, g_fixed, rho_moving, w_moving, g_moving, poses, B, score, grad_pose,
                           grad_w, grad_c, grad_scale, stream);
}

int score_grad_backward(sdf_ctx ctx, const void* rho_fixed, const sdf_grid* g_fixed, const void* rho_moving,
                        const void* w_moving, const sdf_grid* g_moving, const double* poses, int64_t B,
                        const double* grad_score, double* grad_pose, void* grad_w, void* grad_rho_moving,
                        void* grad_rho_fixed, sdf_stream stream) {
    const bool moving_side = grad_pose || grad_w || grad_rho_moving;
    if (!rho_moving || !w_moving || !poses || !grad_score || (moving_side && !rho_fixed))
        return fail(ctx, SDF_EINVAL, "NULL array");
    if (!moving_side && !grad_rho_fixed) return fail(ctx, SDF_EINVAL, "no output requested");
    if (B <= 0) return fail(ctx, SDF_EINVAL, "B must be > 0");
    if (B > (int64_t(1) << 24)) return fail(ctx, SDF_EINVAL, "B too large");
    int rc = check_pair(ctx, g_fixed, g_moving, false);
    if (rc) return rc;
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(ctx, SDF_EHIP, "cannot select device");
    ctx->fused_cache_valid = false;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool planar = g_fixed->n[2] == 1;
    const int N = g_fixed->n[0], nm = g_moving->n[0];
    const int64_t K = gsize(g_moving);
    const size_t el = esize(ctx);
    const int wmode = grad_rho_moving ? 2 : (grad_w ? 1 : 0);
    const size_t gws = ctx->dtype == SDF_F64 ? sdf::grad_workspace_bytes<double>(B, N, nm, planar, wmode)
                                             : sdf::grad_workspace_bytes<float>(B, N, nm, planar, wmode);
    // workspace: the gradient kernels' scratch, the per-pose scores (not
    // returned), the moving coefficients' cotangent; the fixed cotangent's
    // pose table reuses the front once those kernels are done (stream order)
    Carve cv{nullptr};
    cv.take(gws);
    cv.take(el * size_t(B));
    cv.take(2 * el * size_t(K));
    const size_t need = std::max(cv.off, sizeof(double) * 12 * size_t(B) + 256);
    rc = ensure_ws(ctx, need);
    if (rc) return rc;
    Carve c2{static_cast<char*>(ctx->ws)};
    void* gw_ws = c2.take(gws);
    void* score_ws = c2.take(el * size_t(B));
    void* gc = c2.take(2 * el * size_t(K));
    hipError_t e = hipSuccess;
    if (moving_side) {
        void* gcp = grad_rho_moving ? gc : nullptr;
        if (ctx->dtype == SDF_F64)
            e = sdf::launch_score_grad<double>(rho_fixed, N, planar, rho_moving, static_cast<const double*>(w_moving),
                                               nm, poses, B, static_cast<double*>(score_ws), grad_pose,
                                               static_cast<double*>(grad_w), static_cast<double*>(gcp), grad_score,
                                               gw_ws, s);
        else
            e = sdf::launch_score_grad<float>(rho_fixed, N, planar, rho_moving, static_cast<const float*>(w_moving), nm,
                                              poses, B, static_cast<float*>(score_ws), grad_pose,
                                              static_cast<float*>(grad_w), static_cast<float*>(gcp), grad_score,
                                              gw_ws, s);
        if (e == hipSuccess && grad_pose) e = sdf::launch_pose_chain(grad_pose, grad_score, B, grad_pose, s);
        if (e == hipSuccess && grad_rho_moving)
            e = ctx->dtype == SDF_F64
                    ? sdf::launch_rho_from_c<double>(static_cast<const double*>(w_moving), gc, K, grad_rho_moving, s)
                    : sdf::launch_rho_from_c<float>(static_cast<const float*>(w_moving), gc, K, grad_rho_moving, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "score_grad_backward");
    }
    if (grad_rho_fixed) {
        e = ctx->dtype == SDF_F64
                ? sdf::launch_fixed_cotangent<double>(rho_moving, static_cast<const double*>(w_moving), nm, planar, N,
                                                      poses, B, grad_score, grad_rho_fixed, ctx->ws, s)
                : sdf::launch_fixed_cotangent<float>(rho_moving, static_cast<const float*>(w_moving), nm, planar, N,
                                                     poses, B, grad_score, grad_rho_fixed, ctx->ws, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "score_grad_backward");
    }
    return SDF_OK;
}

int score_grad_pose_chain(sdf_ctx ctx, const double* grad_pose, const double* grad_score, int64_t B,
                          double* grad_pose_out, sdf_stream stream) {
    if (!grad_pose || !grad_score || !grad_pose_out) return fail(ctx, SDF_EINVAL, "NULL array");
    if (B <= 0 || B > (int64_t(1) << 24)) return fail(ctx, SDF_EINVAL, "B must be in [1, 2^24]");
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(ctx, SDF_EHIP, "cannot select device");
    hipError_t e = sdf::launch_pose_chain(grad_pose, grad_score, B, grad_pose_out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(ctx, e, "score_grad_pose_chain");
    return SDF_OK;
}

int score_grad_fixed(sdf_ctx ctx, const sdf_grid* g_fixed, const void* rho_moving, const void* w_moving,
                     const sdf_grid* g_moving, const double* poses, int64_t B, const double* grad_scale, void* grad_f,
                     sdf_stream stream) {
    if (!rho_moving || !w_moving || !poses || !grad_f) return fail(ctx, SDF_EINVAL, "NULL array");
    if (B <= 0) return fail(ctx, SDF_EINVAL, "B must be > 0");
    if (B > (int64_t(1) << 24)) return fail(ctx, SDF_EINVAL, "B too large");
    int rc = check_pair(ctx, g_fixed, g_moving, false);
    if (rc) return rc;
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    ctx->fused_cache_valid = false;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool planar = g_fixed->n[2] == 1;
    const int N = g_fixed->n[0], nm = g_moving->n[0];
    rc = ensure_ws(ctx, sizeof(double) * 12 * size_t(B) + 256);
    if (rc) return rc;
    hipError_t e = ctx->dtype == SDF_F64
                       ? sdf::launch_fixed_cotangent<double>(rho_moving, static_cast<const double*>(w_moving), nm,
                                                             planar, N, poses, B, grad_scale, grad_f, ctx->ws, s)
                       : sdf::launch_fixed_cotangent<float>(rho_moving, static_cast<const float*>(w_moving), nm,
                                                            planar, N, poses, B, grad_scale, grad_f, ctx->ws, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "score_grad_fixed");
    return SDF_OK;
}

int octree_samples(sdf_ctx ctx, const void* rho_moving, const void* w_moving, const sdf_grid* g_moving, double tol,
                   int max_level, void* pos_out, void* c_out, int32_t* level_out, int64_t* count_out,
                   sdf_stream stream) {
    if (!rho_moving || !w_moving || !pos_out || !c_out || !count_out) return fail(ctx, SDF_EINVAL, "NULL array");
    int rc = check_grid(ctx, g_moving, "g_moving");
    if (rc) return rc;
    const int nm = g_moving->n[0];
    const bool planar = g_moving->n[2] == 1;
    if (g_moving->n[1] != nm || (!planar && g_moving->n[2] != nm))
        return fail(ctx, SDF_EINVAL, "g_moving: must be N_M^3 or N_M^2 x 1");
    if (nm < 8 || nm % 8) return fail(ctx, SDF_EINVAL, "g_moving: N_M must be a positive multiple of 8");
    if (max_level < 0 || max_level > 3) return fail(ctx, SDF_EINVAL, "max_level must be in [0, 3]");
    if (!std::isfinite(tol) || tol < 0) return fail(ctx, SDF_EINVAL, "tol must be finite and >= 0");
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    ctx->fused_cache_valid = false;
    rc = ensure_ws(ctx, sdf::octree_workspace_bytes(nm, planar, esize(ctx)));
    if (rc) return rc;
    int* lv = reinterpret_cast<int*>(level_out);
    hipError_t e =
        ctx->dtype == SDF_F64
            ? sdf::launch_octree<double>(rho_moving, static_cast<const double*>(w_moving), nm, planar, tol, max_level,
                                         static_cast<double*>(pos_out), c_out, lv, count_out, ctx->ws, s)
            : sdf::launch_octree<float>(rho_moving, static_cast<const float*>(w_moving), nm, planar, tol, max_level,
                                        static_cast<float*>(pos_out), c_out, lv, count_out, ctx->ws, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "octree_samples");
    return SDF_OK;
}

int score_rotations_nfft(sdf_ctx ctx, const void* spec_fixed, const sdf_grid* g_fixed, const void* pos,
                         const void* c, int64_t m, int width, const double* quats, int64_t n_rot, void* peak_score,
                         int32_t* peak_t, void* peak_nbhd, double* refined_t, sdf_stream stream) {
    if (!peak_score || !peak_t) return fail(ctx, SDF_EINVAL, "NULL array");
    int rc = check_nfft_args(ctx, spec_fixed, g_fixed, pos, c, m, width, quats, n_rot);
    if (rc) return rc;
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ctx->dtype == SDF_F64)
        return nfft_impl<double>(ctx, spec_fixed, g_fixed, pos, c, m, width, quats, n_rot, Mode::Peaks, peak_score,
                                 peak_t, peak_nbhd, refined_t, nullptr, s);
    return nfft_impl<float>(ctx, spec_fixed, g_fixed, pos, c, m, width, quats, n_rot, Mode::Peaks, peak_score, peak_t,
                            peak_nbhd, refined_t, nullptr, s);
}

int score_volume_nfft(sdf_ctx ctx, const void* spec_fixed, const sdf_grid* g_fixed, const void* pos, const void* c,
                      int64_t m, int width, const double* quats, int64_t n_rot, void* vol_out, sdf_stream stream) {
    if (!vol_out) return fail(ctx, SDF_EINVAL, "NULL array");
    int rc = check_nfft_args(ctx, spec_fixed, g_fixed, pos, c, m, width, quats, n_rot);
    if (rc) return rc;
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ctx->dtype == SDF_F64)
        return nfft_impl<double>(ctx, spec_fixed, g_fixed, pos, c, m, width, quats, n_rot, Mode::Volume, nullptr,
                                 nullptr, nullptr, nullptr, vol_out, s);
    return nfft_impl<float>(ctx, spec_fixed, g_fixed, pos, c, m, width, quats, n_rot, Mode::Volume, nullptr, nullptr,
                            nullptr, nullptr, vol_out, s);
}

}  // extern "C"
