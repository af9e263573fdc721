// C ABI of the sdfdock library: argument validation, context and workspace
// management, and dispatch to the kernel launchers.  No exception escapes
// any entry point; every failure returns a code and records a message.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <type_traits>
#include <string>
#include <vector>

#include "launch.hpp"
#include "sdfdock.h"

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
    Rec cur;
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
    void begin(const char* name, hipStream_t s) override {
        cur.name = name;
        cur.a = get();
        cur.b = get();
        if (cur.a) (void)hipEventRecord(cur.a, s);
    }
    void end(hipStream_t s) override {
        if (cur.b) (void)hipEventRecord(cur.b, s);
        pending.push_back(cur);
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
    GraphEntry graph;
    Profiler prof;
    int64_t graph_captures = 0;
    int64_t graph_launches = 0;
};

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
    if (need_fft && int(std::ceil(diag)) + 4 > N)
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
struct Layout {
    double* quats;
    double* r64;
    void* rT;
    void* c;
    void* grid;   // plain path: per-rotation complex grid(s)
    void* pval;
    int* pidx;
    void* fused;  // fused path workspace
    size_t total;
};

template <typename T>
Layout carve_search(char* base, int64_t n_rot, int64_t K, int64_t G, int nparts, int plain_batch,
                    const sdf::FusedPlan* fp) {
    Carve cv{base};
    Layout L{};
    L.quats = static_cast<double*>(cv.take(sizeof(double) * 4 * n_rot));
    L.r64 = static_cast<double*>(cv.take(sizeof(double) * 9 * n_rot));
    L.rT = cv.take(sizeof(T) * 9 * n_rot);
    L.c = cv.take(2 * sizeof(T) * K);
    if (fp) {
        L.fused = cv.take(sdf::fused_workspace_bytes(*fp));
        L.grid = nullptr;
        L.pval = nullptr;
        L.pidx = nullptr;
    } else {
        L.grid = cv.take(2 * sizeof(T) * G * plain_batch);
        L.pval = cv.take(sizeof(T) * nparts * plain_batch);
        L.pidx = static_cast<int*>(cv.take(sizeof(int) * nparts * plain_batch));
        L.fused = nullptr;
    }
    L.total = cv.off;
    return L;
}

enum class Mode { Peaks, Volume };

template <typename T>
int search_impl(sdf_ctx ctx, const void* spec, const sdf_grid* gf, const void* rho_m, const void* w_m,
                const sdf_grid* gm, const double* quats, int64_t n_rot, Mode mode, void* score, int32_t* tout,
                void* nbhd, double* refined, void* vol_out, hipStream_t s) {
    const int N = gf->n[0];
    const bool planar = gf->n[2] == 1;
    const int nm = gm->n[0];
    const int64_t K = gsize(gm);
    const int64_t G = gsize(gf);
    const int nparts = sdf::peak_parts<T>(N, planar);
    const bool want_fused = std::is_same<T, float>::value && mode == Mode::Peaks &&
                            (ctx->opt_path == 2 || ctx->opt_path == 0);
    sdf::FusedPlan fp{N, nm, planar, int(ctx->opt_batch), int(ctx->opt_pencil_group)};
    if (want_fused && fp.batch > n_rot) fp.batch = int((n_rot + 1) / 2 * 2);
    const int plain_batch = 1;
    Layout L = carve_search<T>(nullptr, n_rot, K, G, nparts, plain_batch, want_fused ? &fp : nullptr);
    int rc = ensure_ws(ctx, L.total);
    if (rc) return rc;
    L = carve_search<T>(static_cast<char*>(ctx->ws), n_rot, K, G, nparts, plain_batch, want_fused ? &fp : nullptr);

    SDF_TRY_HIP(ctx, hipMemcpyAsync(L.quats, quats, sizeof(double) * 4 * n_rot, hipMemcpyHostToDevice, s),
                "quaternion upload");
    SDF_TRY_HIP(ctx, sdf::launch_quat_to_rot<T>(L.quats, n_rot, L.r64, static_cast<T*>(L.rT), s), "rotations");
    SDF_TRY_HIP(ctx, sdf::launch_coef<T>(rho_m, static_cast<const T*>(w_m), K, L.c, s), "coefficients");

    const T* RT = static_cast<const T*>(L.rT);
    if (want_fused) {
        SDF_TRY_HIP(ctx, sdf::launch_fused_prep(fp, L.c, L.fused, s), "fixed-point scale");
        sdf::KernelTimer* kt = ctx->opt_profile ? &ctx->prof : nullptr;
        auto enqueue = [&]() -> hipError_t {
            for (int64_t r0 = 0; r0 < n_rot; r0 += fp.batch) {
                const int nb = int(n_rot - r0 < fp.batch ? n_rot - r0 : fp.batch);
                hipError_t e = sdf::launch_fused_batch(fp, reinterpret_cast<const float*>(RT) + 9 * r0, nb, L.c, spec,
                                                       L.fused, static_cast<float*>(score) + r0, tout + 3 * r0,
                                                       nbhd ? static_cast<float*>(nbhd) + 27 * r0 : nullptr,
                                                       refined ? refined + 3 * r0 : nullptr, s, kt);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        };
        // Replay a captured graph of the whole launch sequence when the same
        // buffers and shapes come back (capture needs a non-null stream).
        if (ctx->opt_graph && !kt && s != nullptr) {
            std::vector<uintptr_t> key = {uintptr_t(spec), uintptr_t(L.c), uintptr_t(L.rT), uintptr_t(L.fused),
                                          uintptr_t(score), uintptr_t(tout), uintptr_t(nbhd), uintptr_t(refined),
                                          uintptr_t(n_rot), uintptr_t(N), uintptr_t(nm), uintptr_t(planar),
                                          uintptr_t(fp.batch), uintptr_t(fp.pencil_group), uintptr_t(s)};
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
    for (int64_t r = 0; r < n_rot; ++r) {
        SDF_TRY_HIP(ctx, sdf::launch_zero<T>(L.grid, G, s), "zero");
        SDF_TRY_HIP(ctx, sdf::launch_spread_atomic<T>(L.c, nm, planar, RT + 9 * r, 1, T(-1), N, L.grid, s),
                    "spread");
        SDF_TRY_HIP(ctx, sdf::launch_fft3<T>(L.grid, N, planar, 1, -1, 1.0, s), "forward fft");
        SDF_TRY_HIP(ctx, sdf::launch_mul_spec<T>(L.grid, spec, G, 1, s), "spectral product");
        SDF_TRY_HIP(ctx, sdf::launch_fft3<T>(L.grid, N, planar, 1, +1, 1.0, s), "inverse fft");
        if (mode == Mode::Volume) {
            SDF_TRY_HIP(ctx, sdf::launch_real_part<T>(L.grid, static_cast<T*>(vol_out) + r * G, G, s), "real part");
        } else {
            SDF_TRY_HIP(ctx,
                        sdf::launch_peak<T>(L.grid, true, N, planar, 1, static_cast<T*>(L.pval), L.pidx, nparts,
                                            static_cast<T*>(score) + r, tout + 3 * r,
                                            nbhd ? static_cast<T*>(nbhd) + 27 * r : nullptr,
                                            refined ? refined + 3 * r : nullptr, s),
                        "peak");
        }
    }
    return SDF_OK;
}

}  // namespace

// =====================================================================  ABI

extern "C" {

int sdf_ctx_create(sdf_ctx* out, int device, sdf_dtype dtype, size_t workspace_cap_bytes) {
    if (!out) return fail(nullptr, SDF_EINVAL, "out is NULL");
    *out = nullptr;
    if (dtype != SDF_F32 && dtype != SDF_F64) return fail(nullptr, SDF_EINVAL, "unknown dtype");
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
    } else if (!std::strcmp(key, "graph")) {
        if (value != 0 && value != 1) return fail(ctx, SDF_EINVAL, "graph must be 0 or 1");
        ctx->opt_graph = value;
    } else if (!std::strcmp(key, "pencil_group")) {
        if (value != 2 && value != 4) return fail(ctx, SDF_EINVAL, "pencil_group must be 2 or 4");
        ctx->opt_pencil_group = value;
    } else if (!std::strcmp(key, "profile")) {
        if (value != 0 && value != 1) return fail(ctx, SDF_EINVAL, "profile must be 0 or 1");
        ctx->opt_profile = value;
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
    else if (!std::strcmp(key, "graph_captures")) *value = ctx->graph_captures;
    else if (!std::strcmp(key, "graph_launches")) *value = ctx->graph_launches;
    else return fail(ctx, SDF_EINVAL, std::string("unknown option ") + key);
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

int sdf_build(sdf_ctx ctx, const void* q, const void* nrm, const void* w, int64_t n, const sdf_grid* g,
              const sdf_params* p, void* rho_out, sdf_stream stream) {
    if (!q || !nrm || !w || !rho_out) return fail(ctx, SDF_EINVAL, "NULL array");
    if (n <= 0) return fail(ctx, SDF_EINVAL, "sample count must be > 0");
    int rc = check_grid(ctx, g, "grid");
    if (rc) return rc;
    rc = check_params(ctx, p);
    if (rc) return rc;
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(ctx, SDF_EHIP, "cannot select device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const sdf::ParamDesc pd{p->lambda1, p->lambda2, p->sigma, p->eps, p->xi_floor};
    hipError_t e;
    if (ctx->dtype == SDF_F64)
        e = sdf::launch_sdf_build<double>(static_cast<const double*>(q), static_cast<const double*>(nrm),
                                          static_cast<const double*>(w), n, desc(g), pd, rho_out, s);
    else
        e = sdf::launch_sdf_build<float>(static_cast<const float*>(q), static_cast<const float*>(nrm),
                                         static_cast<const float*>(w), n, desc(g), pd, rho_out, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "sdf_build");
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
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ctx->dtype == SDF_F64)
        return search_impl<double>(ctx, spec_fixed, g_fixed, rho_moving, w_moving, g_moving, quats, n_rot,
                                   Mode::Peaks, peak_score, peak_t, peak_nbhd, refined_t, nullptr, s);
    return search_impl<float>(ctx, spec_fixed, g_fixed, rho_moving, w_moving, g_moving, quats, n_rot, Mode::Peaks,
                              peak_score, peak_t, peak_nbhd, refined_t, nullptr, s);
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
    if (ctx->dtype == SDF_F64)
        return search_impl<double>(ctx, spec_fixed, g_fixed, rho_moving, w_moving, g_moving, quats, n_rot,
                                   Mode::Volume, nullptr, nullptr, nullptr, nullptr, vol_out, s);
    return search_impl<float>(ctx, spec_fixed, g_fixed, rho_moving, w_moving, g_moving, quats, n_rot, Mode::Volume,
                              nullptr, nullptr, nullptr, nullptr, vol_out, s);
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
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = ensure_ws(ctx, sdf::topk_workspace_bytes(n));
    if (rc) return rc;
    hipError_t e = ctx->dtype == SDF_F64
                       ? sdf::launch_topk<double>(static_cast<const double*>(scores), n, k, ctx->ws, idx_out, s)
                       : sdf::launch_topk<float>(static_cast<const float*>(scores), n, k, ctx->ws, idx_out, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "topk");
    return SDF_OK;
}

int score_grad(sdf_ctx ctx, const void* rho_fixed, const sdf_grid* g_fixed, const void* rho_moving,
               const void* w_moving, const sdf_grid* g_moving, const double* poses, int64_t B, void* score,
               double* grad_pose, void* grad_w, const double* grad_scale, sdf_stream stream) {
    if (!rho_fixed || !rho_moving || !w_moving || !poses || !score) return fail(ctx, SDF_EINVAL, "NULL array");
    if (B <= 0) return fail(ctx, SDF_EINVAL, "B must be > 0");
    if (B > (int64_t(1) << 24)) return fail(ctx, SDF_EINVAL, "B too large");
    int rc = check_pair(ctx, g_fixed, g_moving, false);
    if (rc) return rc;
    if (!ctx) return fail(nullptr, SDF_EINVAL, "ctx is NULL");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool planar = g_fixed->n[2] == 1;
    const int N = g_fixed->n[0], nm = g_moving->n[0];
    const bool want_w = grad_w != nullptr;
    size_t need = ctx->dtype == SDF_F64 ? sdf::grad_workspace_bytes<double>(B, nm, planar, want_w)
                                        : sdf::grad_workspace_bytes<float>(B, nm, planar, want_w);
    rc = ensure_ws(ctx, need);
    if (rc) return rc;
    hipError_t e;
    if (ctx->dtype == SDF_F64)
        e = sdf::launch_score_grad<double>(rho_fixed, N, planar, rho_moving, static_cast<const double*>(w_moving), nm,
                                           poses, B, static_cast<double*>(score), grad_pose,
                                           static_cast<double*>(grad_w), grad_scale, ctx->ws, s);
    else
        e = sdf::launch_score_grad<float>(rho_fixed, N, planar, rho_moving, static_cast<const float*>(w_moving), nm,
                                          poses, B, static_cast<float*>(score), grad_pose,
                                          static_cast<float*>(grad_w), grad_scale, ctx->ws, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "score_grad");
    return SDF_OK;
}

}  // extern "C"
