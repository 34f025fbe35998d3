// voge_launch.hpp -- host-side launchers of the libvoge kernels and the
// workspace slices they use.  Internal to the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "voge_internal.hpp"

namespace voge {

struct PairRec;

// Device pointers into one caller-owned workspace (see plan_workspace).
struct WsPtrs {
    WsHeader* hdr;
    uint32_t *keys, *vals, *keys2, *vals2, *hist;
    CullRec* cull;
    TraceRec* rec;
    GeoRec* geo;
    float* gM;        // [N][3] camera-space centre gradients, depth-bound order
    float* gS;        // [N][6] camera-space symmetric inverse-covariance gradients
    double* tileD;    // [n_tiles][3] per-tile sums of dL/dD'
    double* camP;     // [n_epi_blocks][12] per-block camera gradient partials
    // per-pixel kept lists, slot-major: [K][S] with S = n_tiles * 256
    int32_t* keff;    // [S]
    double* kl_l;     // depth l (D' units)
    float* kl_m;      // e^q
    float* kl_s;      // sqrt(a)
    float* kl_T;      // transmittance T(l_k)
    int32_t* kl_r;    // rank (depth-bound order)
    int32_t* kl_i;    // original kernel index
    float4* bw;       // backward scratch: per-slot sums over the pair loop
    PairRec* pairs;   // backward scratch: per-tile pair records, kernel-sorted [tiles][256 * K]
};

struct Plan {
    size_t off_keys, off_vals, off_keys2, off_vals2, off_hist, off_cull, off_rec, off_geo;
    size_t off_keff, off_kl_l, off_kl_m, off_kl_s, off_kl_T, off_kl_r, off_kl_i;
    size_t off_gM, off_gS, off_tileD, off_camP, off_bw, off_pairs;
    size_t fwd_bytes, bwd_bytes;
    size_t S;          // list stride: n_tiles * 256
    int n_tiles, n_epi_blocks, sort_blocks;
};

Plan plan_workspace(int N, int C, int H, int W, int K);
WsPtrs carve(void* base, const Plan& p, bool with_backward);
int sort_blocks(int N);

constexpr int EPI_THREADS = 256;

void launch_fill_u32(void* p, size_t n, uint32_t v, hipStream_t s);
void launch_zero3(float* a, size_t na, float* b, size_t nb, float* c, size_t nc, hipStream_t s);
void launch_prep(const float* means, const float* covs, int N, const CamDev& cam, double rad2, const WsPtrs& w,
                 hipStream_t s);

struct TraceArgs {
    WsHeader* hdr;             // status word and tile queue
    int n_cu;                  // compute units (persistent grid size)
    const CullRec* cull;
    const TraceRec* rec;
    const GeoRec* geo;
    int N, H, W, K, C;
    int n_tiles;
    size_t S;                  // list stride
    float F, cx, cy;
    double rad2;               // 2 ln(1/eta) = -2 ln(eta)
    const float* attrs;
    // kept lists
    int32_t* keff;
    double* kl_l;
    float* kl_m;
    float* kl_s;
    float* kl_T;
    int32_t* kl_r;
    int32_t* kl_i;
    // forward outputs
    float* image;
    float* wsum;
    int32_t* kept;
    // backward inputs / outputs
    const float* grad_image;
    float* grad_attrs;
    float* gM;
    float* gS;
    double* tileD;
    float4* bw;
    PairRec* pairs;
};

int pick_kbuf(int K);        // compiled K-buffer depth for a requested K
int table_capacity(int C);   // entries of the per-tile gradient table
size_t bwd_lds_bytes(int hcap, int KB);
hipError_t launch_select(const TraceArgs& a, hipStream_t s);
hipError_t launch_blend(const TraceArgs& a, hipStream_t s);
hipError_t launch_bwd(const TraceArgs& a, hipStream_t s);          // pixel phase
hipError_t launch_bwd_reduce(const TraceArgs& a, hipStream_t s);   // tile reduction
hipError_t launch_phi(const float* x, float* y, int n, hipStream_t s);

struct EpiArgs {
    const float* means;
    const float* covs;
    const TraceRec* rec;
    int N, C;
    CamDev cam;
    const float* gM;
    const float* gS;
    const double* tileD;
    int n_tiles;
    double* camP;
    float* grad_means;
    float* grad_covs;
    float* grad_camera;        // 15 floats or null
};
hipError_t launch_epilogue(const EpiArgs& a, hipStream_t s);

}  // namespace voge
