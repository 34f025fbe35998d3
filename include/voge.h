/*
 * voge.h -- C ABI of libvoge, the rendering hot path of VoGE on AMD MI355X
 * (gfx950, CDNA4).
 *
 * VoGE ("VoGE: A Differentiable Volume Renderer using Gaussian Ellipsoids for
 * Analysis-by-Synthesis", Wang et al., ICLR 2023) renders a set of Gaussian
 * ellipsoid kernels seen by a pinhole camera.  For every pixel ray the library
 *   1. transforms each kernel to camera space (Sec. 3.3, Eq. 3-4),
 *   2. traces it along the ray: peak depth l, log peak density q and the 1D
 *      precision a = 1/sigma^2 (Sec. 3.3, Eq. 5-6; App. A.1),
 *   3. keeps the K nearest kernels (by l) whose peak density e^q exceeds eta,
 *      after a conservative coarse stage on screen tiles (Sec. 3.3
 *      "Coarse-to-fine rendering"; App. A.3),
 *   4. evaluates the closed-form transmittance T(l_k) as an erf sum and the
 *      weights W_k = T(l_k) e^{q_k} (Eq. 7-8; App. A.2), and
 *   5. blends the per-kernel attributes: C = sum_k W_k c_k (Eq. 8).
 * The backward returns gradients w.r.t. the kernels and the camera (the paper
 * states both, Sec. 3.3), with the kept sets held fixed.
 *
 * Conventions
 *   - Array arguments are DEVICE pointers to contiguous, row-major buffers
 *     owned by the caller (float32 unless stated).  Structs passed by pointer
 *     (camera, params) live in HOST memory and are read before return.
 *   - Kernel k: means[k*3 + d]; covariance Sigma_k packed as covs[k*6 + e] in
 *     the order xx, xy, xz, yy, yz, zz (must be symmetric positive definite);
 *     attributes attrs[k*C + c].
 *   - Camera: X_cam = R X + T with R row-major; focal F and principal point
 *     (cx = O_x, cy = O_y) in pixels.  The ray of pixel (i, j), row i and
 *     column j, has direction ((i - O_y)/F, (j - O_x)/F, 1) (Eq. 5).
 *   - Images are HWC: image[(i*W + j)*C + c].
 *   - Absorption tau = 1; the erf argument is (t - l_m) sqrt(a_m) as printed in
 *     Eq. 7; the transmittance sum runs over the kept set, including k; ties in
 *     l are broken by a fixed kernel order; kernels need l > 0; background 0.
 *   - Every call is asynchronous on `stream` (a hipStream_t, 0 = default) and
 *     allocates nothing.  Calls are reentrant across distinct workspaces; two
 *     calls in flight on one workspace race.
 *   - Outputs are overwritten, never accumulated.
 *   - Return value: VOGE_OK, or a negative VOGE_E* code with a message from
 *     voge_last_error().  Host-checked errors leave outputs untouched.
 *   - Conditions found on the device (a covariance that is not SPD, a
 *     non-finite input) do not fail the call: the affected kernel is left out
 *     of the render and gets zero gradient, and a bit is set in the
 *     workspace's status word (voge_status).
 *
 * Limits: 0 <= N < 2^24 kernels, 1 <= C <= 1024 channels, 1 <= H, W <= 32767,
 * 1 <= K <= 64, 0 < eta < 1, F > 0.
 */
#ifndef VOGE_H
#define VOGE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VOGE_OK 0
#define VOGE_EINVAL (-1)      /* bad argument: shape, null pointer, range      */
#define VOGE_ENOSPACE (-2)    /* workspace smaller than voge_workspace_size()  */
#define VOGE_EHIP (-3)        /* a HIP runtime call failed                     */

#define VOGE_STATUS_NOTSPD 1     /* some covariance was not SPD (skipped)      */
#define VOGE_STATUS_NONFINITE 2  /* some centre or covariance was not finite   */

/* Call flags.  voge_render_backward takes VOGE_REUSE_PREP, VOGE_BLOCK_T and
 * VOGE_BLOCK_RHO; voge_sample takes VOGE_REUSE_PREP alone; voge_render_batch
 * takes VOGE_FORWARD with VOGE_BACKWARD or VOGE_SAMPLE or neither, or
 * VOGE_BACKWARD or VOGE_SAMPLE alone, optionally with VOGE_REUSE_PREP
 * (without VOGE_FORWARD), VOGE_GRAPH, VOGE_TUNED and (with VOGE_BACKWARD)
 * the two ablation bits. */
#define VOGE_REUSE_PREP 1     /* the workspace holds the preparation and kept
                                 lists of a forward of the same items          */
#define VOGE_FORWARD 2        /* batch: render the images                      */
#define VOGE_BACKWARD 4       /* batch: gradients of the images                */
#define VOGE_GRAPH 8          /* batch: replay the call's launches from a HIP
                                 graph cached per shape (captured on first use) */
#define VOGE_TUNED 16         /* batch: use the execution choices voge_tune_batch
                                 found for these shapes (defaults if none)     */
#define VOGE_SAMPLE 32        /* batch: sample the feature maps onto the kernels
                                 (Sec. 3.4, Eq. 10; see voge_sample)           */
/* Gradient ablations of the backward (the paper's pose-estimation ablation
 * table), for voge_render_backward and batches with VOGE_BACKWARD: */
#define VOGE_BLOCK_T 64       /* no gradient through the transmittance T(l_k)  */
#define VOGE_BLOCK_RHO 128    /* no gradient through the factor e^{q_k} of Eq. 8
                                 (e^{q_m} inside T keeps its gradient)         */

#define VOGE_MAX_BATCH 4096   /* items per voge_render_batch call              */

typedef struct voge_camera {
    float R[9];               /* world -> camera rotation, row-major           */
    float T[3];               /* translation                                   */
    float focal;              /* F, pixels                                     */
    float cx;                 /* O_x: principal point column                   */
    float cy;                 /* O_y: principal point row                      */
    int32_t height;           /* H                                             */
    int32_t width;            /* W                                             */
} voge_camera_t;

typedef struct voge_params {
    float eta;                /* density threshold: keep kernels with e^q > eta (App. A.3, default 0.01) */
    int32_t K;                /* K' nearest kernels kept per ray (App. A.3, default 20)                 */
} voge_params_t;

typedef struct voge_ctx voge_ctx_t;

/* One render of a batch: a kernel set seen by a camera.  Pointers as in
 * voge_render_forward / voge_render_backward / voge_sample (device memory);
 * buffers that a call does not use may be NULL (attrs too, in a call with
 * VOGE_SAMPLE alone).  C is the channel count of every per-channel array the
 * call uses.  Items may share kernel arrays (many cameras of one scene) but
 * not output buffers. */
typedef struct voge_item {
    const float* means;       /* [N*3]                                          */
    const float* covs;        /* [N*6] packed xx, xy, xz, yy, yz, zz            */
    const float* attrs;       /* [N*C]                                          */
    int32_t N;
    int32_t C;
    voge_camera_t camera;
    voge_params_t params;
    float* image;             /* [H*W*C] out, required with VOGE_FORWARD        */
    float* wsum;              /* [H*W] out, optional                            */
    int32_t* kept;            /* [H*W*K] out, optional                          */
    const float* grad_image;  /* [H*W*C] in, required with VOGE_BACKWARD        */
    float* grad_means;        /* [N*3] out, required with VOGE_BACKWARD         */
    float* grad_covs;         /* [N*6] out, required with VOGE_BACKWARD         */
    float* grad_attrs;        /* [N*C] out, required with VOGE_BACKWARD         */
    float* grad_camera;       /* [15] out, optional                             */
    const float* features;    /* [H*W*C] in, required with VOGE_SAMPLE          */
    float* sampled;           /* [N*C] out, required with VOGE_SAMPLE           */
    float* sample_weight;     /* [N] out, optional                              */
} voge_item_t;

/* Create a library context bound to HIP device `device`.  Host memory only:
 * the context holds a ring of four pinned host buffers (hipHostMalloc, 1.5 MB
 * each) that stage item tables of large batches, the cached HIP graphs and
 * the autotuner's choices; no device memory.  The calls below run on that
 * device (the caller's current device is restored on return).
 * Errors: VOGE_EINVAL (null ctx), VOGE_EHIP. */
int voge_create(voge_ctx_t** ctx, int device);

/* Release a context: waits for its staging copies, frees the pinned buffers
 * and destroys its cached graphs. */
int voge_destroy(voge_ctx_t* ctx);

/* Bytes of workspace needed for N kernels, C channels and this camera's image
 * size; with_backward = 1 sizes it for voge_render_backward and voge_sample as
 * well (the forward uses a prefix of the same layout, so one workspace serves
 * all three).
 * The workspace must be device memory aligned to 256 bytes. */
int voge_workspace_size(int N, int C, const voge_camera_t* cam, const voge_params_t* params, int with_backward,
                        size_t* bytes);

/* Forward render (Sec. 3.3, Eq. 3-8).
 *   image    [H*W*C]  out: C_p = sum_{k in S_p} W_k c_k
 *   wsum     [H*W]    out, optional (NULL): sum_{k in S_p} W_k
 *   kept     [H*W*K]  out, optional (NULL), int32: original indices of the kept
 *                     kernels in ascending l, -1 padded
 *   workspace         device, >= voge_workspace_size(..., 0); afterwards it
 *                     holds this camera's prepared kernels (VOGE_REUSE_PREP). */
int voge_render_forward(voge_ctx_t* ctx, const float* means, const float* covs, const float* attrs, int N, int C,
                        const voge_camera_t* cam, const voge_params_t* params, float* image, float* wsum,
                        int32_t* kept, void* workspace, size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): the forward
 * of voge_render_forward with its workspace in a fixed device array of
 * VOGE_STATIC_WORKSPACE_BYTES that the library holds on each GPU it runs on,
 * from voge_create until the process ends.  Arguments as for
 * voge_render_forward, without the workspace.  Allocates nothing.
 *   Errors: as voge_render_forward; VOGE_ENOSPACE when the render needs more
 *   workspace than the array holds (voge_workspace_size(..., 0) tells the
 *   need; 64 MiB holds e.g. a 512x512 image at K = 8 or 256x256 at K = 20).
 *   Every call on one GPU uses that GPU's one array: calls that overlap on
 *   one GPU (two streams, or two host threads) race, and the device status
 *   word of the call is not readable (voge_status needs a workspace). */
#define VOGE_STATIC_WORKSPACE_BYTES (64u << 20)
int voge_render_forward_static(voge_ctx_t* ctx, const float* means, const float* covs, const float* attrs, int N,
                               int C, const voge_camera_t* cam, const voge_params_t* params, float* image,
                               float* wsum, int32_t* kept, void* stream);

/* Backward of voge_render_forward for upstream gradient grad_image [H*W*C]
 * (the kept sets are held fixed; selection is not differentiable).
 *   grad_means [N*3], grad_covs [N*6] (w.r.t. the 6 packed numbers: each
 *   off-diagonal entry stands for both matrix positions), grad_attrs [N*C]:
 *   all required, overwritten.
 *   grad_camera [15] optional (NULL): dL/dR (9, row-major, entries treated as
 *   independent), dL/dT (3), dL/dF, dL/dO_x, dL/dO_y.
 *   flags: VOGE_REUSE_PREP when `workspace` still holds the preparation done
 *   by voge_render_forward for the same kernels, camera and params (skips it);
 *   VOGE_BLOCK_T / VOGE_BLOCK_RHO for the ablated gradients (attribute
 *   gradients are unchanged by either).
 *   workspace: >= voge_workspace_size(..., 1). */
int voge_render_backward(voge_ctx_t* ctx, const float* means, const float* covs, const float* attrs, int N, int C,
                         const voge_camera_t* cam, const voge_params_t* params, const float* grad_image,
                         float* grad_means, float* grad_covs, float* grad_attrs, float* grad_camera, int flags,
                         void* workspace, size_t workspace_bytes, void* stream);

/* Sampler: the inverse reconstruction of Sec. 3.4 (Eq. 10).  Every kernel
 * takes the W-weighted mean of a feature map phi over the pixels that keep it,
 *   alpha_k = sum_p W_pk phi_p / sum_p W_pk,   W_pk = T(l_k) e^{q_k} (Eq. 8),
 * with the kept sets and weights of voge_render_forward for the same kernels,
 * camera and params.
 *   features       [H*W*C] in: phi, HWC like the images
 *   sampled        [N*C] out: alpha; 0 for a kernel that no pixel keeps (the
 *                  paper leaves that quotient undefined)
 *   sample_weight  [N] out, optional (NULL): sum_p W_pk, 0 where none
 *   flags          VOGE_REUSE_PREP when `workspace` still holds the forward of
 *                  voge_render_forward for the same kernels, camera and params
 *                  (its kept sets and weights are reused), else 0
 *   workspace      >= voge_workspace_size(..., 1)
 * Per kernel, the sums are accumulated in float32 with atomic adds of
 * per-tile partials (their order may vary from call to call).
 * Errors: VOGE_EINVAL, VOGE_ENOSPACE, VOGE_EHIP. */
int voge_sample(voge_ctx_t* ctx, const float* means, const float* covs, int N, int C, const voge_camera_t* cam,
                const voge_params_t* params, const float* features, float* sampled, float* sample_weight, int flags,
                void* workspace, size_t workspace_bytes, void* stream);

/* Exact-integral mode, a diagnostic of the closed form (App. A.2): for every
 * pixel's kept set (the same selection as voge_render_forward) the outer
 * integral of Eq. 1 by quadrature and the closed form of Eq. 7-8, in FP64.
 * Along the ray kernel m has density e^{q_m} g_m(t), g_m(t) =
 * sqrt(a_m/pi) exp(-a_m (t - l_m)^2), whose running integral is the erf sum
 * of Eq. 7; then
 *   W_m = int exp(-E(t)) e^{q_m} g_m(t) dt
 * by the trapezoid rule on n_samples points over
 * [min_m l_m - 9/sqrt(a_m), max_m l_m + 9/sqrt(a_m)].
 *   n_samples  3 .. 2^24 quadrature points per pixel
 *   w_exact    [H*W*K] double out: the quadrature W, kept-list order, 0 padded
 *   w_approx   [H*W*K] double out: the closed form T(l_k) e^{q_k}
 *   total      [H*W*2] double out: sum_k w_exact, and 1 - exp(-sum_m e^{q_m})
 *              (the total mass the closed form reaches in the limit)
 *   kept       [H*W*K] int32 out, optional: the kept kernels, -1 padded
 *   flags      VOGE_REUSE_PREP to take the kept sets of a forward on
 *              `workspace`, else 0
 *   workspace  >= voge_workspace_size(..., 0)
 * Errors: VOGE_EINVAL, VOGE_ENOSPACE, VOGE_EHIP. */
int voge_quadrature(voge_ctx_t* ctx, const float* means, const float* covs, int N, const voge_camera_t* cam,
                    const voge_params_t* params, int n_samples, double* w_exact, double* w_approx, double* total,
                    int32_t* kept, int flags, void* workspace, size_t workspace_bytes, void* stream);

/* Bytes of workspace for a batch of n_items (1 <= n_items <= VOGE_MAX_BATCH);
 * with_backward = 1 sizes it for VOGE_BACKWARD and VOGE_SAMPLE too.  Only
 * the shapes (N, C, camera size, K) of the items matter. */
int voge_batch_workspace_size(const voge_item_t* items, int n_items, int with_backward, size_t* bytes);

/* Render a batch of items in one sequence of launches: every item's kernels
 * are prepared and depth-sorted together, then each stage covers the screen
 * tiles of all items (items with K-buffers of one compiled depth share a
 * launch).  Per item, the results are those of voge_render_forward and
 * voge_render_backward on that item alone, up to the order of floating-point
 * accumulation and the order of kernels at exactly equal depth.
 *   items      host array [n_items], read before return
 *   flags      VOGE_FORWARD, VOGE_BACKWARD, VOGE_SAMPLE, or VOGE_FORWARD with
 *              one of the other two (VOGE_BACKWARD and VOGE_SAMPLE share
 *              scratch and do not combine); VOGE_REUSE_PREP with
 *              VOGE_BACKWARD or VOGE_SAMPLE alone when `workspace` holds a
 *              forward of the same items (shapes, kernels, cameras, params) --
 *              then the kept sets of that forward are used; VOGE_GRAPH replays the launches
 *              from a HIP graph that the context caches per (workspace,
 *              flags, item shapes); it needs a stream other than the null
 *              stream, and the graph is captured on that stream at first use.
 *   workspace  >= voge_batch_workspace_size(items, n_items, VOGE_BACKWARD or
 *              VOGE_SAMPLE set)
 * The item table is staged through the context: two calls on one context may
 * run from different threads, but calls in flight on one workspace race.
 * Errors: VOGE_EINVAL (an item's shapes or pointers, flags), VOGE_ENOSPACE,
 * VOGE_EHIP. */
int voge_render_batch(voge_ctx_t* ctx, const voge_item_t* items, int n_items, int flags, void* workspace,
                      size_t workspace_bytes, void* stream);

/* Autotuner.  For the shapes of a batch (per item: image size, K, C and the
 * bit length of N, in call order; plus the work flags and the device
 * architecture) it times the execution choices -- launches issued one by one
 * or replayed from a HIP graph; the order in which workgroups take screen
 * tiles (a contiguous band of tiles per XCD, for L2 locality, or every eighth
 * tile per XCD, for balance); and which scenes get coarse-stage bins (per
 * 16x16 tile the kernels whose screen box meets it, so that a tile scans its
 * bin instead of every kernel; building them costs a pass over the kernels
 * and a sort per tile) -- on the caller's batch, and keeps the fastest in
 * the context for calls with VOGE_TUNED.  Results are those of
 * voge_render_batch (the call renders the batch 1 + trials times per choice).
 *   flags      as for voge_render_batch, without VOGE_GRAPH and VOGE_TUNED
 *   trials     timed renders per choice (>= 1); graph choices need a non-null stream
 *   result     optional: the choice kept and the mean times (ms) of it and of
 *              the default (separate launches, banded order, no bins)
 * Synchronises `stream`.  Errors as for voge_render_batch. */
typedef struct voge_tune_result {
    int32_t graph;            /* 1 if the kept choice replays a HIP graph      */
    int32_t order;            /* 0 banded tiles per XCD, 1 plain tile order     */
    int32_t bins;             /* coarse-stage bins: 0 none (the default), 1 for
                                 scenes of 16,384 kernels or more, 2 every
                                 scene                                          */
    double best_ms;
    double default_ms;
} voge_tune_result_t;

int voge_tune_batch(voge_ctx_t* ctx, const voge_item_t* items, int n_items, int flags, void* workspace,
                    size_t workspace_bytes, void* stream, int trials, voge_tune_result_t* result);

/* Save the context's tuned choices to `path` (JSON lines: arch, key, graph,
 * order, ms), or merge those of a file written by voge_tune_save; entries of
 * another architecture are skipped on load.  Errors: VOGE_EINVAL (null
 * arguments, unreadable or malformed file). */
int voge_tune_save(voge_ctx_t* ctx, const char* path);
int voge_tune_load(voge_ctx_t* ctx, const char* path);

/* Per-item device status words (VOGE_STATUS_* bits) of the last batch (or
 * single render) on `workspace`, in the caller's item order.  Synchronises
 * `stream`. */
int voge_batch_status(const void* workspace, int n_items, int32_t* device_status, void* stream);

/* Read the workspace's device status word (VOGE_STATUS_* bits of the last
 * forward, or backward without VOGE_REUSE_PREP).  Synchronises `stream`. */
int voge_status(const void* workspace, int32_t* device_status, void* stream);

/* Message of the last error on this thread ("" if none). */
const char* voge_last_error(void);

/* ABI version: major * 10000 + minor * 100 + patch. */
int voge_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VOGE_H */
