// voge_launch.hpp -- host-side launchers of the libvoge kernels, the per-item
// records they read, and the workspace slices they use.  Internal to the
// library.
//
// Every call renders a batch of items (a single-camera call is a batch of
// one).  The items' arrays are concatenated in one workspace: kernel records
// in item order, screen tiles in item order, kept lists per item.  Each item's
// record (ItemDev, in the workspace) holds a TraceArgs view whose pointers are
// already offset to that item's slices, so a workgroup finds its item once and
// then works in item-local tile and rank numbers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "voge_internal.hpp"

namespace voge {

constexpr int EPI_THREADS = 256;
constexpr int PREP_THREADS = 256;
constexpr int MAX_BATCH = 4096;          // items per call
constexpr int INIT_ITEMS = 4;            // item records carried by one init launch's arguments

// One item's view of the workspace, as the trace kernels see it.  Ranks and
// tiles are item-local; every pointer is offset to the item's slice.
struct TraceArgs {
    const CullRec* cull;
    const TraceRec* rec;
    const GeoRec* geo;
    int N, H, W, K, C;
    int n_tiles;
    int grad_mode;             // backward ablation bits: 1 no gradient through T, 2 none through e^q of Eq. 8
    size_t S;                  // list stride: n_tiles * 256
    float F, cx, cy;
    double rad2;               // 2 ln(1/eta) = -2 ln(eta)
    // coarse-stage bins: per tile of the item (item-local tile t) the number
    // of kernels whose screen box meets it and the offset of their ranks in
    // the batch's pair list (global); a tile is binned when its list fits
    // the list's capacity (otherwise select scans every record of the item)
    const uint32_t* tcnt;      // [n_tiles]
    const uint32_t* toff;      // [n_tiles]
    const uint32_t* tlist;     // the batch's pair list (item-local ranks, unordered per tile)
    uint32_t tcap;             // pair list capacity
    int binned;                // 0: the item is not binned (select scans all its records)
    // blocks with candidates: per tile of the item, bit b set when some
    // kernel's screen box meets the tile's 8x8 block b (b = 2 * row half +
    // column half); *tdense set when the image is too large for the count
    // grid in LDS (then every block scans).  Select skips a block with its
    // bit clear.
    const uint32_t* tmask;     // [n_tiles]
    const uint32_t* tdense;    // the item's word
    const float* attrs;
    // kept lists, slot-major [K][S]
    int32_t* keff;             // [S]
    double* kl_l;              // depth l (D' units)
    float* kl_m;               // e^q
    float* kl_s;               // sqrt(a)
    float* kl_T;               // transmittance T(l_k)
    int32_t* kl_r;             // rank (depth-bound order)
    int32_t* kl_i;             // original kernel index
    // forward outputs (caller's; any may be null except where stated)
    float* image;
    float* wsum;
    int32_t* kept;
    // backward, and the sampler of Sec. 3.4 (Eq. 10)
    const float* grad_image;   // per-pixel map reduced onto the kernels: dL/dC, or phi when sampling
    float* gA;                 // [N][C] attribute gradients (sampling: sum_p W phi), original kernel order
    float* gW;                 // [N] sampling: sum_p W, original order (shares gM's storage)
    float* gM;                 // [N][3] camera-space centre gradients, original order
    float* gS;                 // [N][6] camera-space inverse-covariance gradients, original order
    double* tileD;             // [n_tiles][3] per-tile sums of dL/dD'
    float4* bw;                // per-slot backward scalars (dq, dl m-side, da, W), slot-major like the lists
    float* bwl;                // per-slot k-side part of dL/dl, slot-major
};

// Per-item record in the workspace.
struct ItemDev {
    TraceArgs t;
    const float* means;
    const float* covs;
    float* grad_means;         // caller's outputs
    float* grad_covs;
    float* grad_attrs;
    float* grad_camera;        // 15 floats or null
    float* sampled;            // sampling outputs: [N*C] alpha, [N] sum_p W (optional)
    float* sample_weight;
    double* camP;              // [n_epi][12] per-block camera partials
    int* status;               // this item's device status word
    CamDev cam;
    int kern_start;            // first global kernel slot
    int tile_start;            // first global tile
    int pblk_start, n_pblk;    // prep blocks (PREP_THREADS kernels each)
    int epi_start, n_epi;      // epilogue blocks (EPI_THREADS kernels each)
};

// Batch-wide arguments of the per-kernel launches.
struct BatchDev {
    const ItemDev* items;      // [n_items], table order
    int n_items;
    const int* pblk_item;      // [total prep blocks] -> item
    const int* epi_item;       // [total epilogue blocks] -> item
    int item_bits;             // high bits of a sort key that hold the item
    WsHeader* hdr;
    // coarse-stage bins over all items' tiles
    uint32_t* tcnt;            // [total tiles] kernels per tile
    uint32_t* tcur;            // [total tiles] scatter cursors
    uint32_t* toff;            // [total tiles + 1] exclusive scan of tcnt
    uint32_t* tlist;           // [tcap] item-local ranks, grouped by tile
    uint32_t tcap;
    int any_binned;            // some item is binned (else no bins are built)
    // block masks over all items' tiles, then one dense word per item
    // (cleared by k_prep_keys, set by k_block_cover); without masks
    // (masks = 0) k_prep_keys marks every item dense
    uint32_t* tmask;           // [total tiles]
    uint32_t* tdense;          // [n_items]
    int masks;
};

// Kernels from which a batch's items get block masks (its largest item's
// count): below it a block's record scan is a few dozen steps, shorter than
// the mask launch.
constexpr int MASK_MIN_KERNELS = 2048;

// One launch over the tiles of a group of items that share a K-buffer depth.
struct GroupDev {
    const ItemDev* items;
    const int* tile_item;      // [total tiles] -> item
    int single;                // the group's item when it has only one, else -1
    int tile0, n_tiles;        // the group's global tiles
    int order;                 // block -> tile order: 0 banded per XCD, 1 plain
    int bins;                  // some item of the group is binned (select stages bins in LDS)
};

// Outputs of the exact-integral mode (one item): per pixel and kept slot,
// [H*W*K] doubles, and per pixel [H*W*2] totals.
struct QuadOut {
    double* w_exact;
    double* w_approx;
    double* total;
    int32_t* kept;             // optional
    int n_samples;
};

// Execution choices of a call, picked by the autotuner per shape.
struct ExecConfig {
    int graph = 0;             // replay the launches from a cached HIP graph
    int order = 0;             // block -> tile order of the trace kernels
    int bins = 0;              // coarse-stage bins: 0 none, 1 items of BIN_MIN_KERNELS or more, 2 every item
};

// Kernels from which an item's tiles are binned under choice 1.  Bins are
// off by default: on the measured workloads (up to 100,000 kernels per
// scene) building and sorting them cost more than the record scan they save.
constexpr int BIN_MIN_KERNELS = 16384;

inline bool item_binned(const ExecConfig& c, int N) {
    return c.bins == 2 || (c.bins == 1 && N >= BIN_MIN_KERNELS);
}

// Host-side plan of a batch: sizes, table order and workspace offsets.
struct ItemShape {
    int N, C, H, W, K;
};

struct ItemPlan {
    int caller;                // index in the caller's array
    int kb;                    // K-buffer depth
    ItemShape s;
    int n_tiles;
    size_t S;
    int kern_start, tile_start, pblk_start, n_pblk, epi_start, n_epi;
    size_t list_off;           // element offset of the kept lists
    size_t attr_off;           // element offset of the attribute gradients
};

struct GroupPlan {
    int kb;
    int first_item, n_items;
    int tile0, n_tiles;
    int max_c;                 // largest channel count of the group's items
};

struct BatchPlan {
    std::vector<ItemPlan> items;     // table order (grouped by K-buffer depth)
    std::vector<GroupPlan> groups;
    int total_kern = 0, total_tiles = 0, total_pblk = 0, total_epi = 0, max_n = 0;
    size_t total_list = 0, total_attr = 0;
    int item_bits = 0, sort_blocks = 0;
    size_t off_items, off_tile_item, off_pblk_item, off_epi_item;
    size_t off_keys, off_vals, off_keys2, off_vals2, off_hist, off_cull, off_rec, off_geo;
    size_t off_keff, off_kl_l, off_kl_m, off_kl_s, off_kl_T, off_kl_r, off_kl_i;
    size_t off_grads, off_tileD, off_camP, off_bw, off_bwl;
    size_t off_tcnt, off_tcur, off_toff, off_tsum, off_tlist, off_tmask;
    uint32_t tile_cap = 0;     // pair list capacity
    int tscan_blocks = 0;      // blocks of the tile-count scan
    size_t fwd_bytes, bwd_bytes;
};

// Fixed workspace prefix: header, then one status word per caller item.
constexpr size_t OFF_STATUS = 256;
constexpr size_t PREFIX_BYTES = OFF_STATUS + sizeof(int) * MAX_BATCH;

int pick_kbuf(int K);        // compiled K-buffer depth for a requested K
int sort_blocks(int N);
int table_capacity(int C);   // entries of the per-tile gradient table
size_t bwd_lds_bytes(int hcap, int KB, int max_c);

// Items first .. first+count-1: writes their table records from the launch
// arguments (from_args, count <= INIT_ITEMS) or reads them from the table,
// fills the block -> item maps and (clear_status) clears their status words
// and, with clear_header, the header's.
struct InitPack {
    ItemDev it[INIT_ITEMS];
};
void launch_init(const InitPack& pack, int first, int count, bool from_args, ItemDev* table, int* tile_item,
                 int* pblk_item, int* epi_item, WsHeader* hdr, bool clear_status, bool clear_header, hipStream_t s);

void launch_fill_u32(void* p, size_t n, uint32_t v, hipStream_t s);
// Prep (keys, depth sort, records) and the coarse-stage bins: per tile the
// kernels whose screen box meets it (count, scan, scatter).  tsum: the
// scan's block sums, tscan_blocks + 1 words.
void launch_prep(const BatchDev& b, int total_pblk, int total_kern, int max_n, int total_tiles, int tscan_blocks,
                 uint32_t* keys, uint32_t* vals, uint32_t* keys2, uint32_t* vals2, uint32_t* hist, uint32_t* tsum,
                 CullRec* cull, TraceRec* rec, GeoRec* geo, hipStream_t s);
constexpr int TSCAN_BLOCK = 1024;        // tile counts per block of the bin scan
// pair list capacity of a batch: generous for boxes of a few tiles each
inline size_t tile_capacity(size_t total_kern, size_t total_tiles) { return 8 * total_kern + 64 * total_tiles + 1024; }

hipError_t launch_select(const GroupDev& g, int kb, hipStream_t s);
hipError_t launch_blend(const GroupDev& g, int kb, hipStream_t s);
hipError_t launch_bwd(const GroupDev& g, int kb, int max_c, hipStream_t s);   // pixel phase + tile reduction
hipError_t launch_fwdbwd(const GroupDev& g, int kb, int max_c, hipStream_t s);   // blend, then the backward
// blend plus the sampler; max_c: the largest channel count of the group's items
hipError_t launch_blend_sample(const GroupDev& g, int kb, int max_c, hipStream_t s);
hipError_t launch_phi(const float* x, float* y, int n, hipStream_t s);
hipError_t launch_quadrature(const GroupDev& g, int kb, const QuadOut& out, hipStream_t s);   // one item
hipError_t launch_epilogue(const BatchDev& b, int total_epi, hipStream_t s);
hipError_t launch_sample_epilogue(const BatchDev& b, int total_epi, hipStream_t s);

}  // namespace voge
