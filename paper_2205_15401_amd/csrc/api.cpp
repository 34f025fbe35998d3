// api.cpp -- the extern "C" entry points of libvoge: argument checks,
// workspace planning and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "voge.h"
#include "voge_debug.h"
#include "voge_launch.hpp"

struct voge_ctx {
    int device;
    int n_cu;
    // optional per-kernel timing: HIP events recorded around launches
    bool profiling = false;
    struct Pending {
        std::string name;
        hipEvent_t a, b;
    };
    std::mutex mu;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<double, long long>> totals;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

// Makes ctx->device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

bool finite_f(float x) { return std::isfinite(x); }

int check_camera(const voge_camera_t* cam) {
    if (!cam) return fail(VOGE_EINVAL, "camera is null");
    for (int e = 0; e < 9; ++e)
        if (!finite_f(cam->R[e])) return fail(VOGE_EINVAL, "camera R is not finite");
    for (int e = 0; e < 3; ++e)
        if (!finite_f(cam->T[e])) return fail(VOGE_EINVAL, "camera T is not finite");
    if (!finite_f(cam->focal) || !(cam->focal > 0.f)) return fail(VOGE_EINVAL, "focal must be finite and > 0");
    if (!finite_f(cam->cx) || !finite_f(cam->cy)) return fail(VOGE_EINVAL, "principal point is not finite");
    if (cam->height < 1 || cam->width < 1 || cam->height > voge::MAX_IMAGE || cam->width > voge::MAX_IMAGE)
        return fail(VOGE_EINVAL, "image size must be in [1, 32767]");
    return VOGE_OK;
}

int check_common(const voge_ctx_t* ctx, const float* means, const float* covs, const float* attrs, int N, int C,
                 const voge_camera_t* cam, const voge_params_t* params) {
    if (!ctx) return fail(VOGE_EINVAL, "ctx is null");
    if (N < 0 || N >= voge::MAX_KERNELS) return fail(VOGE_EINVAL, "N must be in [0, 2^24)");
    if (C < 1 || C > 1024) return fail(VOGE_EINVAL, "C must be in [1, 1024]");
    if (N > 0 && (!means || !covs || !attrs)) return fail(VOGE_EINVAL, "means, covs and attrs are required");
    if (int rc = check_camera(cam)) return rc;
    if (!params) return fail(VOGE_EINVAL, "params is null");
    if (!(params->eta > 0.f && params->eta < 1.f)) return fail(VOGE_EINVAL, "eta must be in (0, 1)");
    if (params->K < 1 || params->K > voge::MAX_K) return fail(VOGE_EINVAL, "K must be in [1, 64]");
    return VOGE_OK;
}

voge::CamDev to_dev(const voge_camera_t* cam) {
    voge::CamDev d;
    for (int e = 0; e < 9; ++e) d.R[e] = cam->R[e];
    for (int e = 0; e < 3; ++e) d.T[e] = cam->T[e];
    d.F = cam->focal;
    d.cx = cam->cx;
    d.cy = cam->cy;
    d.H = cam->height;
    d.W = cam->width;
    return d;
}

int hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) return fail(VOGE_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return VOGE_OK;
}

hipEvent_t take_event(voge_ctx_t* ctx) {
    if (!ctx->pool.empty()) {
        hipEvent_t e = ctx->pool.back();
        ctx->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Times the launches issued during its lifetime when profiling is on.
struct ProfScope {
    voge_ctx_t* ctx;
    hipStream_t s;
    std::string name;
    hipEvent_t a = nullptr;
    ProfScope(voge_ctx_t* c, const char* n, hipStream_t st) : ctx(c), s(st), name(n) {
        if (!ctx || !ctx->profiling) return;
        std::lock_guard<std::mutex> g(ctx->mu);
        a = take_event(ctx);
        if (a) (void)hipEventRecord(a, s);
    }
    ~ProfScope() {
        if (!a) return;
        std::lock_guard<std::mutex> g(ctx->mu);
        hipEvent_t b = take_event(ctx);
        if (!b) return;
        (void)hipEventRecord(b, s);
        ctx->pending.push_back({name, a, b});
    }
};

}  // namespace

namespace voge {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Plan plan_workspace(int N, int C, int H, int W, int K) {
    (void)C;
    Plan p{};
    size_t off = align256(sizeof(WsHeader));
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t n = N > 0 ? (size_t)N : 1;
    const size_t k = K > 0 ? (size_t)K : 1;
    p.n_tiles = ((H + TILE - 1) / TILE) * ((W + TILE - 1) / TILE);
    p.S = (size_t)p.n_tiles * TILE_THREADS;
    p.sort_blocks = sort_blocks((int)n);
    p.off_keys = take(4 * n);
    p.off_vals = take(4 * n);
    p.off_keys2 = take(4 * n);
    p.off_vals2 = take(4 * n);
    p.off_hist = take(4 * 256 * (size_t)p.sort_blocks);
    p.off_cull = take(sizeof(CullRec) * n);
    p.off_rec = take(sizeof(TraceRec) * n);
    p.off_geo = take(sizeof(GeoRec) * n);
    p.off_keff = take(4 * p.S);
    p.off_kl_l = take(8 * k * p.S);
    p.off_kl_m = take(4 * k * p.S);
    p.off_kl_s = take(4 * k * p.S);
    p.off_kl_T = take(4 * k * p.S);
    p.off_kl_r = take(4 * k * p.S);
    p.off_kl_i = take(4 * k * p.S);
    p.fwd_bytes = off;
    p.n_epi_blocks = (int)((n + EPI_THREADS - 1) / EPI_THREADS);
    p.off_gM = take(sizeof(float) * 3 * n);
    p.off_gS = take(sizeof(float) * 6 * n);
    p.off_tileD = take(sizeof(double) * 3 * (size_t)p.n_tiles);
    p.off_camP = take(sizeof(double) * 12 * (size_t)p.n_epi_blocks);
    p.off_bw = take(16 * k * p.S);
    p.off_pairs = take(32 * k * p.S);    // PairRec
    p.bwd_bytes = off;
    return p;
}

WsPtrs carve(void* base, const Plan& p, bool with_backward) {
    unsigned char* b = static_cast<unsigned char*>(base);
    WsPtrs w{};
    w.hdr = reinterpret_cast<WsHeader*>(b);
    w.keys = reinterpret_cast<uint32_t*>(b + p.off_keys);
    w.vals = reinterpret_cast<uint32_t*>(b + p.off_vals);
    w.keys2 = reinterpret_cast<uint32_t*>(b + p.off_keys2);
    w.vals2 = reinterpret_cast<uint32_t*>(b + p.off_vals2);
    w.hist = reinterpret_cast<uint32_t*>(b + p.off_hist);
    w.cull = reinterpret_cast<CullRec*>(b + p.off_cull);
    w.rec = reinterpret_cast<TraceRec*>(b + p.off_rec);
    w.geo = reinterpret_cast<GeoRec*>(b + p.off_geo);
    w.keff = reinterpret_cast<int32_t*>(b + p.off_keff);
    w.kl_l = reinterpret_cast<double*>(b + p.off_kl_l);
    w.kl_m = reinterpret_cast<float*>(b + p.off_kl_m);
    w.kl_s = reinterpret_cast<float*>(b + p.off_kl_s);
    w.kl_T = reinterpret_cast<float*>(b + p.off_kl_T);
    w.kl_r = reinterpret_cast<int32_t*>(b + p.off_kl_r);
    w.kl_i = reinterpret_cast<int32_t*>(b + p.off_kl_i);
    if (with_backward) {
        w.gM = reinterpret_cast<float*>(b + p.off_gM);
        w.gS = reinterpret_cast<float*>(b + p.off_gS);
        w.tileD = reinterpret_cast<double*>(b + p.off_tileD);
        w.camP = reinterpret_cast<double*>(b + p.off_camP);
        w.bw = reinterpret_cast<float4*>(b + p.off_bw);
        w.pairs = reinterpret_cast<PairRec*>(b + p.off_pairs);
    }
    return w;
}

}  // namespace voge

extern "C" {

int voge_version(void) { return 10000; }

const char* voge_last_error(void) { return g_err.c_str(); }

int voge_create(voge_ctx_t** ctx, int device) {
    if (!ctx) return fail(VOGE_EINVAL, "ctx is null");
    int count = 0;
    if (int rc = hip_check(hipGetDeviceCount(&count), "hipGetDeviceCount")) return rc;
    if (device < 0 || device >= count) return fail(VOGE_EINVAL, "device out of range");
    int n_cu = 0;
    if (int rc = hip_check(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device),
                           "hipDeviceGetAttribute"))
        return rc;
    voge_ctx_t* c = new voge_ctx();
    c->device = device;
    c->n_cu = n_cu;
    *ctx = c;
    g_err.clear();
    return VOGE_OK;
}

int voge_destroy(voge_ctx_t* ctx) {
    if (!ctx) return VOGE_OK;
    {
        std::lock_guard<std::mutex> g(ctx->mu);
        for (auto& p : ctx->pending) {
            (void)hipEventSynchronize(p.b);
            ctx->pool.push_back(p.a);
            ctx->pool.push_back(p.b);
        }
        for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
    }
    delete ctx;
    return VOGE_OK;
}

int voge_workspace_size(int N, int C, const voge_camera_t* cam, const voge_params_t* params, int with_backward,
                        size_t* bytes) {
    if (!bytes) return fail(VOGE_EINVAL, "bytes is null");
    if (N < 0 || N >= voge::MAX_KERNELS) return fail(VOGE_EINVAL, "N must be in [0, 2^24)");
    if (C < 1 || C > 1024) return fail(VOGE_EINVAL, "C must be in [1, 1024]");
    if (int rc = check_camera(cam)) return rc;
    if (!params || params->K < 1 || params->K > voge::MAX_K) return fail(VOGE_EINVAL, "K must be in [1, 64]");
    const voge::Plan p = voge::plan_workspace(N, C, cam->height, cam->width, params->K);
    *bytes = with_backward ? p.bwd_bytes : p.fwd_bytes;
    return VOGE_OK;
}

namespace {

voge::TraceArgs trace_args(const voge_ctx_t* ctx, const voge::WsPtrs& w, const voge::Plan& p, int N, int C,
                           const voge_camera_t* cam, const voge_params_t* params, const float* attrs) {
    voge::TraceArgs ta{};
    ta.hdr = w.hdr;
    ta.n_cu = ctx->n_cu;
    ta.cull = w.cull;
    ta.rec = w.rec;
    ta.geo = w.geo;
    ta.N = N;
    ta.H = cam->height;
    ta.W = cam->width;
    ta.K = params->K;
    ta.C = C;
    ta.n_tiles = p.n_tiles;
    ta.S = p.S;
    ta.F = cam->focal;
    ta.cx = cam->cx;
    ta.cy = cam->cy;
    ta.rad2 = -2.0 * std::log((double)params->eta);
    ta.attrs = attrs;
    ta.keff = w.keff;
    ta.kl_l = w.kl_l;
    ta.kl_m = w.kl_m;
    ta.kl_s = w.kl_s;
    ta.kl_T = w.kl_T;
    ta.kl_r = w.kl_r;
    ta.kl_i = w.kl_i;
    ta.gM = w.gM;
    ta.gS = w.gS;
    ta.tileD = w.tileD;
    ta.bw = w.bw;
    ta.pairs = w.pairs;
    return ta;
}

// prep + sort + select + blend: the whole forward on `s`
int run_forward(voge_ctx_t* ctx, const float* means, const float* covs, const voge_camera_t* cam,
                const voge::WsPtrs& w, voge::TraceArgs ta, hipStream_t s) {
    {
        ProfScope ps(ctx, "prep", s);
        voge::launch_fill_u32(&w.hdr->status, 1, 0u, s);
        voge::launch_prep(means, covs, ta.N, to_dev(cam), ta.rad2, w, s);
    }
    {
        ProfScope ps(ctx, "select", s);
        if (int rc = hip_check(voge::launch_select(ta, s), "select launch")) return rc;
    }
    {
        ProfScope ps(ctx, "blend", s);
        if (int rc = hip_check(voge::launch_blend(ta, s), "blend launch")) return rc;
    }
    return VOGE_OK;
}

}  // namespace

int voge_render_forward(voge_ctx_t* ctx, const float* means, const float* covs, const float* attrs, int N, int C,
                        const voge_camera_t* cam, const voge_params_t* params, float* image, float* wsum,
                        int32_t* kept, void* workspace, size_t workspace_bytes, void* stream) {
    if (int rc = check_common(ctx, means, covs, attrs, N, C, cam, params)) return rc;
    if (!image) return fail(VOGE_EINVAL, "image is required");
    if (!workspace) return fail(VOGE_EINVAL, "workspace is null");
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(VOGE_EINVAL, "workspace must be 256-byte aligned");
    const voge::Plan p = voge::plan_workspace(N, C, cam->height, cam->width, params->K);
    if (workspace_bytes < p.fwd_bytes) return fail(VOGE_ENOSPACE, "workspace too small");
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(VOGE_EHIP, "cannot select the context's device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const voge::WsPtrs w = voge::carve(workspace, p, false);
    voge::TraceArgs ta = trace_args(ctx, w, p, N, C, cam, params, attrs);
    ta.image = image;
    ta.wsum = wsum;
    ta.kept = kept;
    if (int rc = run_forward(ctx, means, covs, cam, w, ta, s)) return rc;
    g_err.clear();
    return VOGE_OK;
}

int voge_render_backward(voge_ctx_t* ctx, const float* means, const float* covs, const float* attrs, int N, int C,
                         const voge_camera_t* cam, const voge_params_t* params, const float* grad_image,
                         float* grad_means, float* grad_covs, float* grad_attrs, float* grad_camera, int flags,
                         void* workspace, size_t workspace_bytes, void* stream) {
    if (int rc = check_common(ctx, means, covs, attrs, N, C, cam, params)) return rc;
    if (!grad_image) return fail(VOGE_EINVAL, "grad_image is required");
    if (N > 0 && (!grad_means || !grad_covs || !grad_attrs))
        return fail(VOGE_EINVAL, "grad_means, grad_covs and grad_attrs are required");
    if (flags & ~VOGE_REUSE_PREP) return fail(VOGE_EINVAL, "unknown flags");
    if (!workspace) return fail(VOGE_EINVAL, "workspace is null");
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(VOGE_EINVAL, "workspace must be 256-byte aligned");
    const voge::Plan p = voge::plan_workspace(N, C, cam->height, cam->width, params->K);
    if (workspace_bytes < p.bwd_bytes) return fail(VOGE_ENOSPACE, "workspace too small");
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(VOGE_EHIP, "cannot select the context's device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const voge::WsPtrs w = voge::carve(workspace, p, true);
    voge::TraceArgs ta = trace_args(ctx, w, p, N, C, cam, params, attrs);
    if (!(flags & VOGE_REUSE_PREP)) {
        if (int rc = run_forward(ctx, means, covs, cam, w, ta, s)) return rc;   // lists and T, no image
    }
    if (N > 0) {
        ProfScope ps(ctx, "zero", s);
        voge::launch_zero3(w.gM, (size_t)N * 3, w.gS, (size_t)N * 6, grad_attrs, (size_t)N * C, s);
    }
    ta.grad_image = grad_image;
    ta.grad_attrs = grad_attrs;
    {
        ProfScope ps(ctx, "bwd", s);
        if (int rc = hip_check(voge::launch_bwd(ta, s), "backward launch")) return rc;
    }
    {
        ProfScope ps(ctx, "bwd_reduce", s);
        if (int rc = hip_check(voge::launch_bwd_reduce(ta, s), "backward reduce launch")) return rc;
    }
    voge::EpiArgs ea{};
    ea.means = means;
    ea.covs = covs;
    ea.rec = w.rec;
    ea.N = N;
    ea.C = C;
    ea.cam = to_dev(cam);
    ea.gM = w.gM;
    ea.gS = w.gS;
    ea.tileD = w.tileD;
    ea.n_tiles = p.n_tiles;
    ea.camP = w.camP;
    ea.grad_means = grad_means;
    ea.grad_covs = grad_covs;
    ea.grad_camera = grad_camera;
    {
        ProfScope ps(ctx, "epilogue", s);
        if (int rc = hip_check(voge::launch_epilogue(ea, s), "epilogue launch")) return rc;
    }
    g_err.clear();
    return VOGE_OK;
}

int voge_profile_enable(voge_ctx_t* ctx, int enable) {
    if (!ctx) return fail(VOGE_EINVAL, "ctx is null");
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->profiling = enable != 0;
    g_err.clear();
    return VOGE_OK;
}

int voge_profile_read(voge_ctx_t* ctx, voge_phase_time_t* out, int max_out, int* n_out, int reset) {
    if (!ctx || !n_out || max_out < 0 || (max_out > 0 && !out)) return fail(VOGE_EINVAL, "bad arguments");
    std::lock_guard<std::mutex> g(ctx->mu);
    for (auto& p : ctx->pending) {
        float ms = 0.f;
        if (int rc = hip_check(hipEventSynchronize(p.b), "hipEventSynchronize")) return rc;
        if (int rc = hip_check(hipEventElapsedTime(&ms, p.a, p.b), "hipEventElapsedTime")) return rc;
        auto& t = ctx->totals[p.name];
        t.first += ms;
        t.second += 1;
        ctx->pool.push_back(p.a);
        ctx->pool.push_back(p.b);
    }
    ctx->pending.clear();
    int n = 0;
    for (const auto& kv : ctx->totals) {
        if (n < max_out) {
            std::memset(&out[n], 0, sizeof(voge_phase_time_t));
            std::strncpy(out[n].name, kv.first.c_str(), sizeof(out[n].name) - 1);
            out[n].total_ms = kv.second.first;
            out[n].count = kv.second.second;
        }
        ++n;
    }
    *n_out = n;
    if (reset) ctx->totals.clear();
    g_err.clear();
    return VOGE_OK;
}

int voge_debug_phi(const float* x, float* y, int n, void* stream) {
    if (n < 0 || (n > 0 && (!x || !y))) return fail(VOGE_EINVAL, "bad arguments");
    if (int rc = hip_check(voge::launch_phi(x, y, n, static_cast<hipStream_t>(stream)), "phi launch")) return rc;
    g_err.clear();
    return VOGE_OK;
}

int voge_status(const void* workspace, int32_t* device_status, void* stream) {
    if (!workspace || !device_status) return fail(VOGE_EINVAL, "workspace and device_status are required");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t st = 0;
    const auto* hdr = static_cast<const voge::WsHeader*>(workspace);
    if (int rc = hip_check(hipMemcpyAsync(&st, &hdr->status, sizeof(int32_t), hipMemcpyDeviceToHost, s),
                           "hipMemcpyAsync"))
        return rc;
    if (int rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize")) return rc;
    *device_status = st;
    g_err.clear();
    return VOGE_OK;
}

}  // extern "C"
