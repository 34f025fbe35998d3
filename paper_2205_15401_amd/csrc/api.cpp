// api.cpp -- the extern "C" entry points of libvoge: argument checks,
// workspace planning and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "voge.h"
#include "voge_debug.h"
#include "voge_launch.hpp"

namespace {

// A fixed ring of pinned host buffers, made at context creation, stages item
// tables too large for launch arguments.
constexpr int RING_SLOTS = 4;
constexpr int GRAPH_CACHE = 32;

struct Stage {
    void* host = nullptr;
    hipEvent_t done = nullptr;
    bool used = false;
};

struct GraphEntry {
    std::vector<int64_t> key;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};

}  // namespace

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
    // batch tables and graphs
    std::mutex stage_mu;
    std::vector<Stage> ring;
    int ring_next = 0;
    size_t stage_bytes = 0;
    std::mutex graph_mu;
    std::vector<GraphEntry> graphs;
    uint64_t tick = 0;
    // autotuned execution choices per shape key
    std::string arch;
    std::mutex tune_mu;
    std::map<std::string, std::pair<voge::ExecConfig, double>> tuned;
    // this device's copy of the static workspace (voge_render_forward_static)
    void* scratch = nullptr;
    // bin choice of calls without a tuned choice (voge_debug_bins)
    int bins = 0;
};

// The workspace of voge_render_forward_static: a fixed array in device
// memory, one copy on every GPU the library runs on, held until the process
// ends.  On the host the array's name is only a stand-in for the symbol:
// kernels and copies get the device address that hipGetSymbolAddress
// returns for the current device (scratch_address), never the name.
static __device__ __align__(256) unsigned char scratch[VOGE_STATIC_WORKSPACE_BYTES];

namespace {

thread_local std::string g_err;

// Device -> address of its copy of `scratch`, looked up once per device.
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;

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

// attrs == nullptr with need_attrs false: a call that does not read them (the sampler).
int check_common(const voge_ctx_t* ctx, const float* means, const float* covs, const float* attrs, int N, int C,
                 const voge_camera_t* cam, const voge_params_t* params, bool need_attrs = true) {
    if (!ctx) return fail(VOGE_EINVAL, "ctx is null");
    if (N < 0 || N >= voge::MAX_KERNELS) return fail(VOGE_EINVAL, "N must be in [0, 2^24)");
    if (C < 1 || C > 1024) return fail(VOGE_EINVAL, "C must be in [1, 1024]");
    if (N > 0 && (!means || !covs)) return fail(VOGE_EINVAL, "means and covs are required");
    if (N > 0 && need_attrs && !attrs) return fail(VOGE_EINVAL, "attrs is required");
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

// The address of `scratch` on `device` (which must be current): looked up
// with hipGetSymbolAddress the first time, then kept.
int scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it == g_scratch_addr.end()) {
        void* ptr = nullptr;
        if (int rc = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress (scratch)"))
            return rc;
        if (!ptr) return fail(VOGE_EHIP, "hipGetSymbolAddress (scratch) returned null");
        it = g_scratch_addr.emplace(device, ptr).first;
    }
    *out = it->second;
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

// Sizes, table order and workspace layout of a batch.  Items are grouped by
// K-buffer depth (stable), so each group's tiles are contiguous.
BatchPlan plan_batch(const ItemShape* shapes, int n) {
    BatchPlan p;
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return pick_kbuf(shapes[a].K) < pick_kbuf(shapes[b].K); });
    p.items.resize(n);
    for (int j = 0; j < n; ++j) {
        ItemPlan& it = p.items[j];
        it.caller = order[j];
        it.s = shapes[order[j]];
        it.kb = pick_kbuf(it.s.K);
        it.n_tiles = ((it.s.H + TILE - 1) / TILE) * ((it.s.W + TILE - 1) / TILE);
        it.S = (size_t)it.n_tiles * TILE_THREADS;
        it.kern_start = p.total_kern;
        it.tile_start = p.total_tiles;
        it.pblk_start = p.total_pblk;
        it.n_pblk = (it.s.N + PREP_THREADS - 1) / PREP_THREADS;
        it.epi_start = p.total_epi;
        it.n_epi = (it.s.N + EPI_THREADS - 1) / EPI_THREADS;
        it.list_off = p.total_list;
        it.attr_off = p.total_attr;
        p.total_kern += it.s.N;
        p.max_n = std::max(p.max_n, it.s.N);
        p.total_tiles += it.n_tiles;
        p.total_pblk += it.n_pblk;
        p.total_epi += it.n_epi;
        p.total_list += (size_t)it.s.K * it.S;
        p.total_attr += (size_t)it.s.N * it.s.C;
        if (p.groups.empty() || p.groups.back().kb != it.kb)
            p.groups.push_back({it.kb, j, 0, it.tile_start, 0, 1});
        p.groups.back().n_items += 1;
        p.groups.back().max_c = std::max(p.groups.back().max_c, it.s.C);
        p.groups.back().n_tiles += it.n_tiles;
    }
    int ib = 0;
    while ((1 << ib) < n) ++ib;
    p.item_bits = ib;

    size_t off = align256(PREFIX_BYTES);
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t nk = p.total_kern > 0 ? (size_t)p.total_kern : 1;
    const size_t nl = p.total_list > 0 ? p.total_list : 1;
    const size_t nt = p.total_tiles > 0 ? (size_t)p.total_tiles : 1;
    p.sort_blocks = sort_blocks((int)nk);
    p.off_items = take(sizeof(ItemDev) * (size_t)(n > 0 ? n : 1));
    p.off_tile_item = take(sizeof(int) * nt);
    p.off_pblk_item = take(sizeof(int) * (size_t)(p.total_pblk > 0 ? p.total_pblk : 1));
    p.off_epi_item = take(sizeof(int) * (size_t)(p.total_epi > 0 ? p.total_epi : 1));
    p.off_keys = take(4 * nk);
    p.off_vals = take(4 * nk);
    p.off_keys2 = take(4 * nk);
    p.off_vals2 = take(4 * nk);
    p.off_hist = take(4 * 256 * ((size_t)p.sort_blocks + 1));     // block counts per digit, then digit totals
    p.off_cull = take(sizeof(CullRec) * nk);
    p.off_rec = take(sizeof(TraceRec) * nk);
    p.off_geo = take(sizeof(GeoRec) * nk);
    p.off_keff = take(4 * nt * TILE_THREADS);
    p.off_kl_l = take(8 * nl);
    p.off_kl_m = take(4 * nl);
    p.off_kl_s = take(4 * nl);
    p.off_kl_T = take(4 * nl);
    p.off_kl_r = take(4 * nl);
    p.off_kl_i = take(4 * nl);
    p.tile_cap = (uint32_t)std::min<size_t>(tile_capacity(nk, nt), 0xFFFFFFF0u);
    p.tscan_blocks = (int)((nt + TSCAN_BLOCK - 1) / TSCAN_BLOCK);
    p.off_tcnt = take(4 * nt);
    p.off_tcur = take(4 * nt);
    p.off_toff = take(4 * (nt + 1));
    p.off_tsum = take(4 * ((size_t)p.tscan_blocks + 1));
    p.off_tlist = take(4 * (size_t)p.tile_cap);
    p.off_tmask = take(4 * (nt + (size_t)(n > 0 ? n : 1)));    // block masks, then the items' dense words
    p.fwd_bytes = off;
    // gM [3 nk] | gS [6 nk] | gA [total_attr]: one contiguous range, cleared at once
    p.off_grads = take(sizeof(float) * (9 * nk + p.total_attr));
    p.off_tileD = take(sizeof(double) * 3 * nt);
    p.off_camP = take(sizeof(double) * 12 * (size_t)(p.total_epi > 0 ? p.total_epi : 1));
    p.off_bw = take(16 * nl);
    p.off_bwl = take(4 * nl);
    p.bwd_bytes = off;
    return p;
}

}  // namespace voge

namespace {

int validate_item(const voge_item_t& it, int flags, int i) {
    auto bad = [&](const char* what) { return fail(VOGE_EINVAL, "item " + std::to_string(i) + ": " + what); };
    if (it.N < 0 || it.N >= voge::MAX_KERNELS) return bad("N must be in [0, 2^24)");
    if (it.C < 1 || it.C > 1024) return bad("C must be in [1, 1024]");
    if (it.N > 0 && (!it.means || !it.covs)) return bad("means and covs are required");
    if (it.N > 0 && (flags & (VOGE_FORWARD | VOGE_BACKWARD)) && !it.attrs)
        return bad("attrs is required with VOGE_FORWARD or VOGE_BACKWARD");
    if (int rc = check_camera(&it.camera)) return bad(g_err.c_str()), rc;
    if (!(it.params.eta > 0.f && it.params.eta < 1.f)) return bad("eta must be in (0, 1)");
    if (it.params.K < 1 || it.params.K > voge::MAX_K) return bad("K must be in [1, 64]");
    if ((flags & VOGE_FORWARD) && !it.image) return bad("image is required with VOGE_FORWARD");
    if (flags & VOGE_BACKWARD) {
        if (!it.grad_image) return bad("grad_image is required with VOGE_BACKWARD");
        if (it.N > 0 && (!it.grad_means || !it.grad_covs || !it.grad_attrs))
            return bad("grad_means, grad_covs and grad_attrs are required with VOGE_BACKWARD");
    }
    if (flags & VOGE_SAMPLE) {
        if (!it.features) return bad("features is required with VOGE_SAMPLE");
        if (it.N > 0 && !it.sampled) return bad("sampled is required with VOGE_SAMPLE");
    }
    return VOGE_OK;
}

// The work flags of a batch call: at least one of forward, backward and
// sampling; backward and sampling share the gradient scratch; a reused
// preparation excludes a new forward.
int check_work_flags(int flags) {
    if (!(flags & (VOGE_FORWARD | VOGE_BACKWARD | VOGE_SAMPLE)))
        return fail(VOGE_EINVAL, "VOGE_FORWARD, VOGE_BACKWARD or VOGE_SAMPLE is required");
    if ((flags & VOGE_BACKWARD) && (flags & VOGE_SAMPLE))
        return fail(VOGE_EINVAL, "VOGE_BACKWARD and VOGE_SAMPLE do not combine in one call");
    if ((flags & VOGE_REUSE_PREP) && (flags & VOGE_FORWARD))
        return fail(VOGE_EINVAL, "VOGE_REUSE_PREP goes with VOGE_BACKWARD or VOGE_SAMPLE alone");
    if ((flags & (VOGE_BLOCK_T | VOGE_BLOCK_RHO)) && !(flags & VOGE_BACKWARD))
        return fail(VOGE_EINVAL, "VOGE_BLOCK_T and VOGE_BLOCK_RHO go with VOGE_BACKWARD");
    return VOGE_OK;
}

constexpr int WORK_FLAGS =
    VOGE_FORWARD | VOGE_BACKWARD | VOGE_SAMPLE | VOGE_REUSE_PREP | VOGE_BLOCK_T | VOGE_BLOCK_RHO;

voge::ItemShape shape_of(const voge_item_t& it) {
    return {it.N, it.C, it.camera.height, it.camera.width, it.params.K};
}

// Carved device pointers of a batch workspace.
struct BatchWs {
    unsigned char* base;
    voge::WsHeader* hdr;
    int* status;
    voge::ItemDev* items;
    int *tile_item, *pblk_item, *epi_item;
    uint32_t *keys, *vals, *keys2, *vals2, *hist;
    voge::CullRec* cull;
    voge::TraceRec* rec;
    voge::GeoRec* geo;
    int32_t* keff;
    double* kl_l;
    float *kl_m, *kl_s, *kl_T;
    int32_t *kl_r, *kl_i;
    float* grads;
    double* tileD;
    double* camP;
    float4* bw;
    float* bwl;
    uint32_t *tcnt, *tcur, *toff, *tsum, *tlist, *tmask;
};

BatchWs carve_batch(void* ws, const voge::BatchPlan& p) {
    unsigned char* b = static_cast<unsigned char*>(ws);
    BatchWs w{};
    w.base = b;
    w.hdr = reinterpret_cast<voge::WsHeader*>(b);
    w.status = reinterpret_cast<int*>(b + voge::OFF_STATUS);
    w.items = reinterpret_cast<voge::ItemDev*>(b + p.off_items);
    w.tile_item = reinterpret_cast<int*>(b + p.off_tile_item);
    w.pblk_item = reinterpret_cast<int*>(b + p.off_pblk_item);
    w.epi_item = reinterpret_cast<int*>(b + p.off_epi_item);
    w.keys = reinterpret_cast<uint32_t*>(b + p.off_keys);
    w.vals = reinterpret_cast<uint32_t*>(b + p.off_vals);
    w.keys2 = reinterpret_cast<uint32_t*>(b + p.off_keys2);
    w.vals2 = reinterpret_cast<uint32_t*>(b + p.off_vals2);
    w.hist = reinterpret_cast<uint32_t*>(b + p.off_hist);
    w.cull = reinterpret_cast<voge::CullRec*>(b + p.off_cull);
    w.rec = reinterpret_cast<voge::TraceRec*>(b + p.off_rec);
    w.geo = reinterpret_cast<voge::GeoRec*>(b + p.off_geo);
    w.keff = reinterpret_cast<int32_t*>(b + p.off_keff);
    w.kl_l = reinterpret_cast<double*>(b + p.off_kl_l);
    w.kl_m = reinterpret_cast<float*>(b + p.off_kl_m);
    w.kl_s = reinterpret_cast<float*>(b + p.off_kl_s);
    w.kl_T = reinterpret_cast<float*>(b + p.off_kl_T);
    w.kl_r = reinterpret_cast<int32_t*>(b + p.off_kl_r);
    w.kl_i = reinterpret_cast<int32_t*>(b + p.off_kl_i);
    w.grads = reinterpret_cast<float*>(b + p.off_grads);
    w.tileD = reinterpret_cast<double*>(b + p.off_tileD);
    w.camP = reinterpret_cast<double*>(b + p.off_camP);
    w.bw = reinterpret_cast<float4*>(b + p.off_bw);
    w.bwl = reinterpret_cast<float*>(b + p.off_bwl);
    w.tcnt = reinterpret_cast<uint32_t*>(b + p.off_tcnt);
    w.tcur = reinterpret_cast<uint32_t*>(b + p.off_tcur);
    w.toff = reinterpret_cast<uint32_t*>(b + p.off_toff);
    w.tsum = reinterpret_cast<uint32_t*>(b + p.off_tsum);
    w.tlist = reinterpret_cast<uint32_t*>(b + p.off_tlist);
    w.tmask = reinterpret_cast<uint32_t*>(b + p.off_tmask);
    return w;
}

// The device record of table entry j.
voge::ItemDev item_record(const voge::BatchPlan& p, int j, const voge_item_t& src, const BatchWs& w, int flags,
                          const voge::ExecConfig& cfg) {
    const voge::ItemPlan& ip = p.items[j];
    voge::ItemDev d{};
    voge::TraceArgs& t = d.t;
    const size_t k0 = (size_t)ip.kern_start, lo = ip.list_off;
    t.cull = w.cull + k0;
    t.rec = w.rec + k0;
    t.geo = w.geo + k0;
    t.N = ip.s.N;
    t.H = ip.s.H;
    t.W = ip.s.W;
    t.K = ip.s.K;
    t.C = ip.s.C;
    t.n_tiles = ip.n_tiles;
    t.grad_mode = ((flags & VOGE_BLOCK_T) ? 1 : 0) | ((flags & VOGE_BLOCK_RHO) ? 2 : 0);
    t.S = ip.S;
    t.F = src.camera.focal;
    t.cx = src.camera.cx;
    t.cy = src.camera.cy;
    t.rad2 = -2.0 * std::log((double)src.params.eta);
    t.tcnt = w.tcnt + ip.tile_start;
    t.toff = w.toff + ip.tile_start;
    t.tlist = w.tlist;
    t.tcap = p.tile_cap;
    t.binned = voge::item_binned(cfg, ip.s.N) ? 1 : 0;
    t.tmask = w.tmask + ip.tile_start;
    t.tdense = w.tmask + (p.total_tiles > 0 ? p.total_tiles : 1) + j;
    t.attrs = src.attrs;
    t.keff = w.keff + (size_t)ip.tile_start * voge::TILE_THREADS;
    t.kl_l = w.kl_l + lo;
    t.kl_m = w.kl_m + lo;
    t.kl_s = w.kl_s + lo;
    t.kl_T = w.kl_T + lo;
    t.kl_r = w.kl_r + lo;
    t.kl_i = w.kl_i + lo;
    if (flags & VOGE_FORWARD) {
        t.image = src.image;
        t.wsum = src.wsum;
        t.kept = src.kept;
    }
    if (flags & VOGE_SAMPLE) {
        const size_t nk = p.total_kern > 0 ? (size_t)p.total_kern : 1;
        float* gM = w.grads;
        float* gA = gM + 9 * nk;
        t.grad_image = src.features;
        t.gW = gM + 3 * k0;
        t.gA = gA + ip.attr_off;
        d.sampled = src.sampled;
        d.sample_weight = src.sample_weight;
    }
    if (flags & VOGE_BACKWARD) {
        const size_t nk = p.total_kern > 0 ? (size_t)p.total_kern : 1;
        float* gM = w.grads;
        float* gS = gM + 3 * nk;
        float* gA = gS + 6 * nk;
        t.grad_image = src.grad_image;
        t.gM = gM + 3 * k0;
        t.gS = gS + 6 * k0;
        t.gA = gA + ip.attr_off;
        t.tileD = w.tileD + 3 * (size_t)ip.tile_start;
        t.bw = w.bw + lo;
        t.bwl = w.bwl + lo;
        d.grad_means = src.grad_means;
        d.grad_covs = src.grad_covs;
        d.grad_attrs = src.grad_attrs;
        d.grad_camera = src.grad_camera;
        d.camP = w.camP + 12 * (size_t)ip.epi_start;
    }
    d.means = src.means;
    d.covs = src.covs;
    d.status = w.status + ip.caller;
    d.cam = to_dev(&src.camera);
    d.kern_start = ip.kern_start;
    d.tile_start = ip.tile_start;
    d.pblk_start = ip.pblk_start;
    d.n_pblk = ip.n_pblk;
    d.epi_start = ip.epi_start;
    d.n_epi = ip.n_epi;
    return d;
}

voge::BatchDev batch_dev(const voge::BatchPlan& p, const BatchWs& w, const voge::ExecConfig& cfg) {
    voge::BatchDev b{};
    for (const auto& it : p.items) b.any_binned |= voge::item_binned(cfg, it.s.N) ? 1 : 0;
    b.items = w.items;
    b.n_items = (int)p.items.size();
    b.pblk_item = w.pblk_item;
    b.epi_item = w.epi_item;
    b.item_bits = p.item_bits;
    b.hdr = w.hdr;
    b.tcnt = w.tcnt;
    b.tcur = w.tcur;
    b.toff = w.toff;
    b.tlist = w.tlist;
    b.tcap = p.tile_cap;
    b.tmask = w.tmask;
    b.tdense = w.tmask + (p.total_tiles > 0 ? p.total_tiles : 1);
    b.masks = p.max_n >= voge::MASK_MIN_KERNELS ? 1 : 0;
    return b;
}

voge::GroupDev group_dev(const voge::BatchPlan& p, const voge::GroupPlan& g, const BatchWs& w,
                         const voge::ExecConfig& cfg) {
    voge::GroupDev d{};
    d.items = w.items;
    d.tile_item = w.tile_item;
    d.single = g.n_items == 1 ? g.first_item : -1;
    d.tile0 = g.tile0;
    d.n_tiles = g.n_tiles;
    d.order = cfg.order;
    for (int j = g.first_item; j < g.first_item + g.n_items; ++j) d.bins |= voge::item_binned(cfg, p.items[j].s.N) ? 1 : 0;
    return d;
}

// Writes the item table into the workspace: through launch arguments for a
// few items, else through a pinned staging buffer of the context's ring.
int upload_items(voge_ctx_t* ctx, const std::vector<voge::ItemDev>& recs, const BatchWs& w, bool clear_status,
                 hipStream_t s);

// All launches of a call after the table upload.
int launch_compute(voge_ctx_t* ctx, const voge::BatchPlan& p, const BatchWs& w, int flags,
                   const voge::ExecConfig& cfg, bool profile, hipStream_t s, const voge::QuadOut* quad = nullptr) {
    const voge::BatchDev b = batch_dev(p, w, cfg);
    auto scope = [&](const char* name) { return ProfScope(profile ? ctx : nullptr, name, s); };
    const bool fwd_part = (flags & VOGE_FORWARD) || !(flags & VOGE_REUSE_PREP);
    if (fwd_part) {
        {
            ProfScope ps = scope("prep");
            voge::launch_prep(b, p.total_pblk, p.total_kern, p.max_n, p.total_tiles, p.tscan_blocks, w.keys, w.vals,
                              w.keys2, w.vals2, w.hist, w.tsum, w.cull, w.rec, w.geo, s);
            if (int rc = hip_check(hipGetLastError(), "prep launch")) return rc;
        }
        {
            ProfScope ps = scope("select");
            for (const auto& g : p.groups)
                if (int rc = hip_check(voge::launch_select(group_dev(p, g, w, cfg), g.kb, s), "select launch")) return rc;
        }
    }
    if (quad) {
        // exact-integral mode (one item): the quadrature replaces the blend
        ProfScope ps = scope("quadrature");
        const voge::GroupPlan& g = p.groups[0];
        return hip_check(voge::launch_quadrature(group_dev(p, g, w, cfg), g.kb, *quad, s), "quadrature launch");
    }
    if (flags & VOGE_SAMPLE) {
        {
            ProfScope ps = scope("zero");
            const size_t nk = p.total_kern > 0 ? (size_t)p.total_kern : 1;
            voge::launch_fill_u32(w.grads, 9 * nk + p.total_attr, 0u, s);
        }
        {
            // the blend, with the sampler's per-tile reduction fused in
            ProfScope ps = scope("blend_sample");
            for (const auto& g : p.groups)
                if (int rc = hip_check(voge::launch_blend_sample(group_dev(p, g, w, cfg), g.kb, g.max_c, s),
                                       "blend+sample launch"))
                    return rc;
        }
        {
            ProfScope ps = scope("sample_epilogue");
            if (int rc = hip_check(voge::launch_sample_epilogue(b, p.total_epi, s), "sample epilogue launch"))
                return rc;
        }
    } else if (fwd_part && (flags & VOGE_FORWARD) && (flags & VOGE_BACKWARD)) {
        // forward and backward in one call: the blend and the backward run
        // in one kernel per K-buffer group
        {
            ProfScope ps = scope("zero");
            const size_t nk = p.total_kern > 0 ? (size_t)p.total_kern : 1;
            voge::launch_fill_u32(w.grads, 9 * nk + p.total_attr, 0u, s);
        }
        {
            ProfScope ps = scope("fwdbwd");
            for (const auto& g : p.groups)
                if (int rc = hip_check(voge::launch_fwdbwd(group_dev(p, g, w, cfg), g.kb, g.max_c, s), "fwd+bwd launch"))
                    return rc;
        }
        ProfScope ps = scope("epilogue");
        return hip_check(voge::launch_epilogue(b, p.total_epi, s), "epilogue launch");
    } else if (fwd_part) {
        ProfScope ps = scope("blend");
        for (const auto& g : p.groups)
            if (int rc = hip_check(voge::launch_blend(group_dev(p, g, w, cfg), g.kb, s), "blend launch")) return rc;
    }
    if (flags & VOGE_BACKWARD) {
        {
            ProfScope ps = scope("zero");
            const size_t nk = p.total_kern > 0 ? (size_t)p.total_kern : 1;
            voge::launch_fill_u32(w.grads, 9 * nk + p.total_attr, 0u, s);
        }
        {
            ProfScope ps = scope("bwd");
            for (const auto& g : p.groups)
                if (int rc = hip_check(voge::launch_bwd(group_dev(p, g, w, cfg), g.kb, g.max_c, s), "backward launch"))
                    return rc;
        }
        {
            ProfScope ps = scope("epilogue");
            if (int rc = hip_check(voge::launch_epilogue(b, p.total_epi, s), "epilogue launch")) return rc;
        }
    }
    return VOGE_OK;
}

std::vector<int64_t> graph_key(const voge::BatchPlan& p, const void* ws, int flags, const voge::ExecConfig& cfg) {
    std::vector<int64_t> k;
    k.reserve(4 + 5 * p.items.size());
    k.push_back((int64_t)reinterpret_cast<uintptr_t>(ws));
    k.push_back(flags & WORK_FLAGS);
    k.push_back(cfg.order);
    k.push_back(cfg.bins);
    k.push_back((int64_t)p.items.size());
    for (const auto& it : p.items) {
        k.push_back(it.caller);
        k.push_back(it.s.N);
        k.push_back(it.s.C);
        k.push_back(((int64_t)it.s.H << 32) | (uint32_t)it.s.W);
        k.push_back(it.s.K);
    }
    return k;
}

int run_graph(voge_ctx_t* ctx, const voge::BatchPlan& p, const BatchWs& w, int flags, const voge::ExecConfig& cfg,
              hipStream_t s);

// The autotuner's key of a call: the device architecture, the work flags and
// the items' shapes in call order (height x width, K, C and the bit length of
// N), run-length coded.
std::string shape_key(const voge_ctx_t* ctx, const voge_item_t* items, int n, int flags) {
    std::string k = ctx->arch + ";f" + std::to_string(flags & WORK_FLAGS) + ";";
    std::string prev;
    int run = 0;
    auto flush = [&]() {
        if (run > 0) k += prev + "*" + std::to_string(run) + ",";
    };
    for (int i = 0; i < n; ++i) {
        int nb = 0;
        while ((1LL << nb) <= (long long)items[i].N) ++nb;
        const std::string sh = std::to_string(items[i].camera.height) + "x" + std::to_string(items[i].camera.width) +
                               "/K" + std::to_string(items[i].params.K) + "/C" + std::to_string(items[i].C) + "/N" +
                               std::to_string(nb);
        if (sh != prev) {
            flush();
            prev = sh;
            run = 0;
        }
        ++run;
    }
    flush();
    return k;
}

// The whole call: checks, plan, table, launches.  `force` overrides the
// execution choices (the autotuner's trials).
int run_batch(voge_ctx_t* ctx, const voge_item_t* items, int n, int flags, void* workspace, size_t workspace_bytes,
              hipStream_t s, const voge::ExecConfig* force = nullptr, const voge::QuadOut* quad = nullptr) {
    const bool scratch = (flags & (VOGE_BACKWARD | VOGE_SAMPLE)) != 0;   // the gradient scratch is in use
    std::vector<voge::ItemShape> shapes(n);
    for (int i = 0; i < n; ++i) shapes[i] = shape_of(items[i]);
    const voge::BatchPlan p = voge::plan_batch(shapes.data(), n);
    if (p.total_kern >= (1 << 30)) return fail(VOGE_EINVAL, "too many kernels in one batch");
    if (workspace_bytes < (scratch ? p.bwd_bytes : p.fwd_bytes)) return fail(VOGE_ENOSPACE, "workspace too small");
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(VOGE_EHIP, "cannot select the context's device");
    const BatchWs w = carve_batch(workspace, p);
    voge::ExecConfig cfg;
    cfg.bins = ctx->bins;
    if (force) {
        cfg = *force;
    } else {
        if (flags & VOGE_TUNED) {
            const std::string key = shape_key(ctx, items, n, flags);
            std::lock_guard<std::mutex> g(ctx->tune_mu);
            auto it = ctx->tuned.find(key);
            if (it != ctx->tuned.end()) cfg = it->second.first;
        }
        if (flags & VOGE_GRAPH) cfg.graph = 1;
    }
    if (s == nullptr || quad) cfg.graph = 0;       // graphs: non-null streams, render calls only
    std::vector<voge::ItemDev> recs(n);
    for (int j = 0; j < n; ++j) recs[j] = item_record(p, j, items[p.items[j].caller], w, flags, cfg);
    const bool fwd_part = (flags & VOGE_FORWARD) || !(flags & VOGE_REUSE_PREP);
    {
        ProfScope ps(ctx, "upload", s);
        if (int rc = upload_items(ctx, recs, w, fwd_part, s)) return rc;
    }
    if (cfg.graph) return run_graph(ctx, p, w, flags, cfg, s);
    return launch_compute(ctx, p, w, flags, cfg, true, s, quad);
}

}  // namespace

namespace {

int upload_items(voge_ctx_t* ctx, const std::vector<voge::ItemDev>& recs, const BatchWs& w, bool clear_status,
                 hipStream_t s) {
    const int n = (int)recs.size();
    if (n <= 2 * voge::INIT_ITEMS) {
        for (int first = 0; first < n; first += voge::INIT_ITEMS) {
            voge::InitPack pack{};
            const int count = std::min(voge::INIT_ITEMS, n - first);
            for (int b = 0; b < count; ++b) pack.it[b] = recs[first + b];
            voge::launch_init(pack, first, count, true, w.items, w.tile_item, w.pblk_item, w.epi_item, w.hdr,
                              clear_status, clear_status && first == 0, s);
            if (int rc = hip_check(hipGetLastError(), "init launch")) return rc;
        }
        return VOGE_OK;
    }
    const size_t bytes = sizeof(voge::ItemDev) * (size_t)n;
    std::lock_guard<std::mutex> g(ctx->stage_mu);
    if (ctx->ring.empty() || bytes > ctx->stage_bytes) return fail(VOGE_EINVAL, "item table exceeds the staging area");
    Stage& st = ctx->ring[ctx->ring_next];
    ctx->ring_next = (ctx->ring_next + 1) % (int)ctx->ring.size();
    if (st.used) {
        if (int rc = hip_check(hipEventSynchronize(st.done), "hipEventSynchronize (staging)")) return rc;
    }
    std::memcpy(st.host, recs.data(), bytes);
    if (int rc = hip_check(hipMemcpyAsync(w.items, st.host, bytes, hipMemcpyHostToDevice, s), "hipMemcpyAsync (items)"))
        return rc;
    if (int rc = hip_check(hipEventRecord(st.done, s), "hipEventRecord (staging)")) return rc;
    st.used = true;
    voge::InitPack none{};
    voge::launch_init(none, 0, n, false, w.items, w.tile_item, w.pblk_item, w.epi_item, w.hdr, clear_status,
                      clear_status, s);
    return hip_check(hipGetLastError(), "init launch");
}

// Replays the call's launches from a cached graph, capturing it on `s` the
// first time this (workspace, flags, shapes) key is seen.
int run_graph(voge_ctx_t* ctx, const voge::BatchPlan& p, const BatchWs& w, int flags, const voge::ExecConfig& cfg,
              hipStream_t s) {
    const std::vector<int64_t> key = graph_key(p, w.base, flags, cfg);
    std::lock_guard<std::mutex> g(ctx->graph_mu);
    GraphEntry* hit = nullptr;
    for (auto& e : ctx->graphs)
        if (e.key == key) hit = &e;
    if (!hit) {
        if (int rc = hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture"))
            return rc;
        const int rc_launch = launch_compute(ctx, p, w, flags, cfg, false, s);
        hipGraph_t graph = nullptr;
        const hipError_t e_end = hipStreamEndCapture(s, &graph);
        if (rc_launch) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc_launch;
        }
        if (int rc = hip_check(e_end, "hipStreamEndCapture")) return rc;
        hipGraphExec_t exec = nullptr;
        const hipError_t e_inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (int rc = hip_check(e_inst, "hipGraphInstantiate")) return rc;
        if ((int)ctx->graphs.size() >= GRAPH_CACHE) {
            auto lru = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                        [](const GraphEntry& a, const GraphEntry& b) { return a.last_use < b.last_use; });
            (void)hipGraphExecDestroy(lru->exec);
            ctx->graphs.erase(lru);
        }
        ctx->graphs.push_back({key, exec, 0});
        hit = &ctx->graphs.back();
    }
    hit->last_use = ++ctx->tick;
    ProfScope ps(ctx, "graph", s);
    return hip_check(hipGraphLaunch(hit->exec, s), "hipGraphLaunch");
}

voge_item_t single_item(const float* means, const float* covs, const float* attrs, int N, int C,
                        const voge_camera_t* cam, const voge_params_t* params) {
    voge_item_t it{};
    it.means = means;
    it.covs = covs;
    it.attrs = attrs;
    it.N = N;
    it.C = C;
    it.camera = *cam;
    it.params = *params;
    return it;
}

int check_workspace(void* workspace) {
    if (!workspace) return fail(VOGE_EINVAL, "workspace is null");
    if (reinterpret_cast<uintptr_t>(workspace) & 255) return fail(VOGE_EINVAL, "workspace must be 256-byte aligned");
    return VOGE_OK;
}

}  // namespace

extern "C" {

int voge_version(void) { return 10300; }

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
    DeviceGuard guard(device);
    if (!guard.ok) return fail(VOGE_EHIP, "cannot select the device");
    hipDeviceProp_t prop;
    if (int rc = hip_check(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties")) return rc;
    voge_ctx_t* c = new voge_ctx();
    c->device = device;
    c->n_cu = n_cu;
    c->arch = prop.gcnArchName;
    c->arch = c->arch.substr(0, c->arch.find(':'));
    if (int rc = scratch_address(device, &c->scratch)) {
        delete c;
        return rc;
    }
    c->stage_bytes = sizeof(voge::ItemDev) * (size_t)voge::MAX_BATCH;
    c->ring.resize(RING_SLOTS);
    for (auto& st : c->ring) {
        hipError_t e = hipHostMalloc(&st.host, c->stage_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&st.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            voge_destroy(c);
            return hip_check(e, "staging allocation");
        }
    }
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
    {
        std::lock_guard<std::mutex> g(ctx->stage_mu);
        for (auto& st : ctx->ring) {
            if (st.done) {
                if (st.used) (void)hipEventSynchronize(st.done);
                (void)hipEventDestroy(st.done);
            }
            if (st.host) (void)hipHostFree(st.host);
        }
    }
    {
        std::lock_guard<std::mutex> g(ctx->graph_mu);
        for (auto& e : ctx->graphs) (void)hipGraphExecDestroy(e.exec);
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
    const voge::ItemShape sh{N, C, cam->height, cam->width, params->K};
    const voge::BatchPlan p = voge::plan_batch(&sh, 1);
    *bytes = with_backward ? p.bwd_bytes : p.fwd_bytes;
    g_err.clear();
    return VOGE_OK;
}

int voge_render_forward(voge_ctx_t* ctx, const float* means, const float* covs, const float* attrs, int N, int C,
                        const voge_camera_t* cam, const voge_params_t* params, float* image, float* wsum,
                        int32_t* kept, void* workspace, size_t workspace_bytes, void* stream) {
    if (int rc = check_common(ctx, means, covs, attrs, N, C, cam, params)) return rc;
    if (!image) return fail(VOGE_EINVAL, "image is required");
    if (int rc = check_workspace(workspace)) return rc;
    voge_item_t it = single_item(means, covs, attrs, N, C, cam, params);
    it.image = image;
    it.wsum = wsum;
    it.kept = kept;
    if (int rc = run_batch(ctx, &it, 1, VOGE_FORWARD, workspace, workspace_bytes, static_cast<hipStream_t>(stream)))
        return rc;
    g_err.clear();
    return VOGE_OK;
}

int voge_render_forward_static(voge_ctx_t* ctx, const float* means, const float* covs, const float* attrs, int N,
                               int C, const voge_camera_t* cam, const voge_params_t* params, float* image,
                               float* wsum, int32_t* kept, void* stream) {
    if (int rc = check_common(ctx, means, covs, attrs, N, C, cam, params)) return rc;
    if (!image) return fail(VOGE_EINVAL, "image is required");
    if (!ctx->scratch) return fail(VOGE_EHIP, "the context has no static workspace");
    const voge::ItemShape sh{N, C, cam->height, cam->width, params->K};
    const size_t need = voge::plan_batch(&sh, 1).fwd_bytes;
    if (need > (size_t)VOGE_STATIC_WORKSPACE_BYTES)
        return fail(VOGE_ENOSPACE, "the render needs " + std::to_string(need) +
                                       " bytes of workspace, more than the static workspace's " +
                                       std::to_string((size_t)VOGE_STATIC_WORKSPACE_BYTES));
    voge_item_t it = single_item(means, covs, attrs, N, C, cam, params);
    it.image = image;
    it.wsum = wsum;
    it.kept = kept;
    if (int rc = run_batch(ctx, &it, 1, VOGE_FORWARD, ctx->scratch, (size_t)VOGE_STATIC_WORKSPACE_BYTES,
                           static_cast<hipStream_t>(stream)))
        return rc;
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
    if (flags & ~(VOGE_REUSE_PREP | VOGE_BLOCK_T | VOGE_BLOCK_RHO)) return fail(VOGE_EINVAL, "unknown flags");
    if (int rc = check_workspace(workspace)) return rc;
    voge_item_t it = single_item(means, covs, attrs, N, C, cam, params);
    it.grad_image = grad_image;
    it.grad_means = grad_means;
    it.grad_covs = grad_covs;
    it.grad_attrs = grad_attrs;
    it.grad_camera = grad_camera;
    if (int rc = run_batch(ctx, &it, 1, VOGE_BACKWARD | flags, workspace, workspace_bytes,
                           static_cast<hipStream_t>(stream)))
        return rc;
    g_err.clear();
    return VOGE_OK;
}

int voge_sample(voge_ctx_t* ctx, const float* means, const float* covs, int N, int C, const voge_camera_t* cam,
                const voge_params_t* params, const float* features, float* sampled, float* sample_weight, int flags,
                void* workspace, size_t workspace_bytes, void* stream) {
    if (int rc = check_common(ctx, means, covs, nullptr, N, C, cam, params, false)) return rc;
    if (!features) return fail(VOGE_EINVAL, "features is required");
    if (N > 0 && !sampled) return fail(VOGE_EINVAL, "sampled is required");
    if (flags & ~VOGE_REUSE_PREP) return fail(VOGE_EINVAL, "unknown flags");
    if (int rc = check_workspace(workspace)) return rc;
    voge_item_t it = single_item(means, covs, nullptr, N, C, cam, params);
    it.features = features;
    it.sampled = sampled;
    it.sample_weight = sample_weight;
    if (int rc = run_batch(ctx, &it, 1, VOGE_SAMPLE | (flags & VOGE_REUSE_PREP), workspace, workspace_bytes,
                           static_cast<hipStream_t>(stream)))
        return rc;
    g_err.clear();
    return VOGE_OK;
}

int voge_quadrature(voge_ctx_t* ctx, const float* means, const float* covs, int N, const voge_camera_t* cam,
                    const voge_params_t* params, int n_samples, double* w_exact, double* w_approx, double* total,
                    int32_t* kept, int flags, void* workspace, size_t workspace_bytes, void* stream) {
    if (int rc = check_common(ctx, means, covs, nullptr, N, 1, cam, params, false)) return rc;
    if (!w_exact || !w_approx || !total) return fail(VOGE_EINVAL, "w_exact, w_approx and total are required");
    if (n_samples < 3 || n_samples > (1 << 24)) return fail(VOGE_EINVAL, "n_samples must be in [3, 2^24]");
    if (flags & ~VOGE_REUSE_PREP) return fail(VOGE_EINVAL, "unknown flags");
    if (int rc = check_workspace(workspace)) return rc;
    voge_item_t it = single_item(means, covs, nullptr, N, 1, cam, params);
    const voge::QuadOut q{w_exact, w_approx, total, kept, n_samples};
    // the preparation and selection of a forward (unless reused), then the
    // quadrature in place of the blend; the item has no image
    const int work = (flags & VOGE_REUSE_PREP) ? VOGE_REUSE_PREP : VOGE_FORWARD;
    if (int rc = run_batch(ctx, &it, 1, work, workspace, workspace_bytes, static_cast<hipStream_t>(stream), nullptr,
                           &q))
        return rc;
    g_err.clear();
    return VOGE_OK;
}

int voge_batch_workspace_size(const voge_item_t* items, int n_items, int with_backward, size_t* bytes) {
    if (!bytes) return fail(VOGE_EINVAL, "bytes is null");
    if (!items || n_items < 1 || n_items > voge::MAX_BATCH) return fail(VOGE_EINVAL, "n_items must be in [1, 4096]");
    std::vector<voge::ItemShape> shapes(n_items);
    for (int i = 0; i < n_items; ++i) {
        if (int rc = validate_item(items[i], 0, i)) return rc;
        shapes[i] = shape_of(items[i]);
    }
    const voge::BatchPlan p = voge::plan_batch(shapes.data(), n_items);
    *bytes = with_backward ? p.bwd_bytes : p.fwd_bytes;
    g_err.clear();
    return VOGE_OK;
}

int voge_render_batch(voge_ctx_t* ctx, const voge_item_t* items, int n_items, int flags, void* workspace,
                      size_t workspace_bytes, void* stream) {
    if (!ctx) return fail(VOGE_EINVAL, "ctx is null");
    if (!items || n_items < 1 || n_items > voge::MAX_BATCH) return fail(VOGE_EINVAL, "n_items must be in [1, 4096]");
    if (flags & ~(WORK_FLAGS | VOGE_GRAPH | VOGE_TUNED)) return fail(VOGE_EINVAL, "unknown flags");
    if (int rc = check_work_flags(flags)) return rc;
    if ((flags & VOGE_GRAPH) && stream == nullptr) return fail(VOGE_EINVAL, "VOGE_GRAPH needs a non-null stream");
    if (int rc = check_workspace(workspace)) return rc;
    for (int i = 0; i < n_items; ++i)
        if (int rc = validate_item(items[i], flags, i)) return rc;
    if (int rc = run_batch(ctx, items, n_items, flags, workspace, workspace_bytes, static_cast<hipStream_t>(stream)))
        return rc;
    g_err.clear();
    return VOGE_OK;
}

int voge_tune_batch(voge_ctx_t* ctx, const voge_item_t* items, int n_items, int flags, void* workspace,
                    size_t workspace_bytes, void* stream, int trials, voge_tune_result_t* result) {
    if (!ctx) return fail(VOGE_EINVAL, "ctx is null");
    if (!items || n_items < 1 || n_items > voge::MAX_BATCH) return fail(VOGE_EINVAL, "n_items must be in [1, 4096]");
    if (flags & ~WORK_FLAGS) return fail(VOGE_EINVAL, "unknown flags");
    if (int rc = check_work_flags(flags)) return rc;
    if (trials < 1) return fail(VOGE_EINVAL, "trials must be >= 1");
    if (int rc = check_workspace(workspace)) return rc;
    for (int i = 0; i < n_items; ++i)
        if (int rc = validate_item(items[i], flags, i)) return rc;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(VOGE_EHIP, "cannot select the context's device");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<voge::ExecConfig> cands;
    for (int graph = 0; graph < (s ? 2 : 1); ++graph)
        for (int order = 0; order < 2; ++order)
            for (int bins = 0; bins < 3; ++bins) {
                voge::ExecConfig c;
                c.graph = graph;
                c.order = order;
                c.bins = bins;
                cands.push_back(c);
            }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (int rc = hip_check(hipEventCreate(&e0), "hipEventCreate")) return rc;
    if (int rc = hip_check(hipEventCreate(&e1), "hipEventCreate")) {
        (void)hipEventDestroy(e0);
        return rc;
    }
    int rc = VOGE_OK;
    double best = 0.0, dflt = 0.0;
    voge::ExecConfig best_cfg;
    for (size_t ci = 0; ci < cands.size() && rc == VOGE_OK; ++ci) {
        rc = run_batch(ctx, items, n_items, flags, workspace, workspace_bytes, s, &cands[ci]);   // warm-up / capture
        if (rc == VOGE_OK) rc = hip_check(hipEventRecord(e0, s), "hipEventRecord");
        for (int t = 0; t < trials && rc == VOGE_OK; ++t)
            rc = run_batch(ctx, items, n_items, flags, workspace, workspace_bytes, s, &cands[ci]);
        if (rc == VOGE_OK) rc = hip_check(hipEventRecord(e1, s), "hipEventRecord");
        if (rc == VOGE_OK) rc = hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.f;
        if (rc == VOGE_OK) rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        if (rc != VOGE_OK) break;
        const double mean = ms / trials;
        if (ci == 0) dflt = mean;
        if (ci == 0 || mean < best) {
            best = mean;
            best_cfg = cands[ci];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != VOGE_OK) return rc;
    {
        std::lock_guard<std::mutex> g(ctx->tune_mu);
        ctx->tuned[shape_key(ctx, items, n_items, flags)] = {best_cfg, best};
    }
    if (result) {
        result->graph = best_cfg.graph;
        result->order = best_cfg.order;
        result->bins = best_cfg.bins;
        result->best_ms = best;
        result->default_ms = dflt;
    }
    g_err.clear();
    return VOGE_OK;
}

namespace {

// The value after `"name":` in a JSON line written by voge_tune_save.
bool json_field(const std::string& line, const char* name, std::string& out) {
    const std::string tag = std::string("\"") + name + "\":";
    const size_t p = line.find(tag);
    if (p == std::string::npos) return false;
    size_t i = p + tag.size();
    if (i < line.size() && line[i] == '"') {
        const size_t e = line.find('"', i + 1);
        if (e == std::string::npos) return false;
        out = line.substr(i + 1, e - i - 1);
        return true;
    }
    size_t e = i;
    while (e < line.size() && line[e] != ',' && line[e] != '}') ++e;
    out = line.substr(i, e - i);
    return !out.empty();
}

}  // namespace

int voge_tune_save(voge_ctx_t* ctx, const char* path) {
    if (!ctx || !path) return fail(VOGE_EINVAL, "ctx and path are required");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(VOGE_EINVAL, std::string("cannot write ") + path);
    std::lock_guard<std::mutex> g(ctx->tune_mu);
    for (const auto& kv : ctx->tuned) {
        if (kv.first.find('"') != std::string::npos) continue;
        std::fprintf(f, "{\"arch\":\"%s\",\"key\":\"%s\",\"graph\":%d,\"order\":%d,\"bins\":%d,\"ms\":%.6g}\n",
                     ctx->arch.c_str(), kv.first.c_str(), kv.second.first.graph, kv.second.first.order,
                     kv.second.first.bins, kv.second.second);
    }
    const bool ok = std::fclose(f) == 0;
    if (!ok) return fail(VOGE_EINVAL, std::string("cannot write ") + path);
    g_err.clear();
    return VOGE_OK;
}

int voge_tune_load(voge_ctx_t* ctx, const char* path) {
    if (!ctx || !path) return fail(VOGE_EINVAL, "ctx and path are required");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(VOGE_EINVAL, std::string("cannot read ") + path);
    std::map<std::string, std::pair<voge::ExecConfig, double>> got;
    char buf[65536];
    int lineno = 0;
    bool bad = false;
    while (std::fgets(buf, sizeof(buf), f)) {
        ++lineno;
        std::string line(buf);
        while (!line.empty() && (line.back() == '\n' || line.back() == '\r')) line.pop_back();
        if (line.empty()) continue;
        std::string arch, key, graph, order, bins = "0", ms;
        if (!json_field(line, "arch", arch) || !json_field(line, "key", key) || !json_field(line, "graph", graph) ||
            !json_field(line, "order", order) || !json_field(line, "ms", ms)) {
            bad = true;
            break;
        }
        (void)json_field(line, "bins", bins);     // absent in files of earlier versions: the default
        char* end = nullptr;
        const long gv = std::strtol(graph.c_str(), &end, 10);
        if (*end || (gv != 0 && gv != 1)) { bad = true; break; }
        const long ov = std::strtol(order.c_str(), &end, 10);
        if (*end || (ov != 0 && ov != 1)) { bad = true; break; }
        const long bv = std::strtol(bins.c_str(), &end, 10);
        if (*end || bv < 0 || bv > 2) { bad = true; break; }
        const double mv = std::strtod(ms.c_str(), &end);
        if (*end) { bad = true; break; }
        if (arch != ctx->arch) continue;
        voge::ExecConfig c;
        c.graph = (int)gv;
        c.order = (int)ov;
        c.bins = (int)bv;
        got[key] = {c, mv};
    }
    std::fclose(f);
    if (bad) return fail(VOGE_EINVAL, std::string("malformed line ") + std::to_string(lineno) + " in " + path);
    {
        std::lock_guard<std::mutex> g(ctx->tune_mu);
        for (auto& kv : got) ctx->tuned[kv.first] = kv.second;
    }
    g_err.clear();
    return VOGE_OK;
}

int voge_batch_status(const void* workspace, int n_items, int32_t* device_status, void* stream) {
    if (!workspace || !device_status) return fail(VOGE_EINVAL, "workspace and device_status are required");
    if (n_items < 1 || n_items > voge::MAX_BATCH) return fail(VOGE_EINVAL, "n_items must be in [1, 4096]");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const auto* src = static_cast<const unsigned char*>(workspace) + voge::OFF_STATUS;
    if (int rc = hip_check(hipMemcpyAsync(device_status, src, sizeof(int32_t) * (size_t)n_items,
                                          hipMemcpyDeviceToHost, s),
                           "hipMemcpyAsync"))
        return rc;
    if (int rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize")) return rc;
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

int voge_debug_bins(voge_ctx_t* ctx, int bins) {
    if (!ctx) return fail(VOGE_EINVAL, "ctx is null");
    if (bins < 0 || bins > 2) return fail(VOGE_EINVAL, "bins must be 0, 1 or 2");
    ctx->bins = bins;
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
