// prep.hip -- per-kernel preparation for one camera (FP64), and the radix
// sort that puts kernels in ascending order of their depth bound.
//
// Viewing transform (VoGE Sec. 3.3, Eq. 3-4): M = R M0 + T, S = R S0 R^T with
// S0 = Sigma^-1.  Coarse stage (Sec. 3.3 "Coarse-to-fine rendering", App. A.3):
// the paper rasterises a per-ellipsoid screen box at reduced resolution; here
// the box is the exact silhouette bound of the eta-ellipsoid
// {X : (X-M)^T S (X-M) <= 2 ln(1/eta)}, which contains the peak of every ray
// whose peak density e^q exceeds eta, so the coarse stage never changes the
// result.
#include "voge_internal.hpp"
#include "voge_launch.hpp"

namespace voge {

// Lower bound of the camera depth of the eta-ellipsoid, divided by F: no ray
// D' = (u, v, F) can have a passing peak at a ray parameter below it.
__device__ __forceinline__ double depth_bound(double Mz, double Szz, double rad2, double F) {
    return (Mz - sqrt(rad2 * Szz)) / F;
}

__device__ __forceinline__ bool load_kernel(const float* __restrict__ means, const float* __restrict__ covs, int n,
                                            double M0[3], double Sig[6]) {
    bool ok = true;
    const auto m = gp(means) + 3 * (size_t)n;
    const auto c = gp(covs) + 6 * (size_t)n;
    for (int d = 0; d < 3; ++d) {
        M0[d] = (double)m[d];
        ok = ok && isfinite(M0[d]);
    }
    for (int e = 0; e < 6; ++e) {
        Sig[e] = (double)c[e];
        ok = ok && isfinite(Sig[e]);
    }
    return ok;
}

// Sort key of a kernel: the item in the high `ib` bits, then the top bits of
// the depth bound's order key.  Within an item the order is by depth bucket;
// bucket_floor gives the smallest depth bound of a bucket, which is what the
// early exit compares against (every later kernel of the item has a bound at
// least that large).  With ib = 0 the bucket is the bound itself.
__device__ __forceinline__ uint32_t batch_key(uint32_t key32, int item, int ib) {
    return ib ? (((uint32_t)item << (32 - ib)) | (key32 >> ib)) : key32;
}

__device__ __forceinline__ float bucket_floor(uint32_t key, int ib) {
    const uint32_t ok = key << ib;            // depth prefix, low bits cleared
    const uint32_t u = (ok & 0x80000000u) ? (ok & 0x7FFFFFFFu) : ~ok;
    return __uint_as_float(u);
}

__device__ __forceinline__ int item_of_block(const int* __restrict__ map, int n_items) {
    return n_items == 1 ? 0 : map[blockIdx.x];
}

__global__ __launch_bounds__(PREP_THREADS) void k_prep_keys(BatchDev B, uint32_t* __restrict__ keys,
                                                             uint32_t* __restrict__ vals) {
    const int item = item_of_block(B.pblk_item, B.n_items);
    const ItemDev& it = B.items[item];
    const int n = (blockIdx.x - it.pblk_start) * PREP_THREADS + threadIdx.x;
    // the item's block masks start clear (k_block_cover sets them), or the
    // item is dense when the batch has no masks (an item without kernels has
    // no prep block, and select finds no record to scan)
    if (B.masks)
        for (int t = n; t < it.t.n_tiles; t += it.n_pblk * PREP_THREADS) B.tmask[it.tile_start + t] = 0u;
    if (n == 0) B.tdense[item] = B.masks ? 0u : 1u;
    if (n >= it.t.N) return;
    double M0[3], Sig[6], S0[6];
    uint32_t key = KEY_CULLED;
    const bool finite = load_kernel(it.means, it.covs, n, M0, Sig);
    int st = 0;
    if (!finite) {
        st = ST_NONFINITE;
    } else if (!spd_inverse6(Sig, S0)) {
        st = ST_NOTSPD;
    } else {
        const CamDev& cam = it.cam;
        const double r0 = cam.R[6], r1 = cam.R[7], r2 = cam.R[8];
        const double Mz = r0 * M0[0] + r1 * M0[1] + r2 * M0[2] + (double)cam.T[2];
        const double Szz = r0 * (r0 * Sig[0] + r1 * Sig[1] + r2 * Sig[2]) +
                           r1 * (r0 * Sig[1] + r1 * Sig[3] + r2 * Sig[4]) +
                           r2 * (r0 * Sig[2] + r1 * Sig[4] + r2 * Sig[5]);
        const double zhi = Mz + sqrt(it.t.rad2 * Szz);
        if (zhi > 0.0) key = float_order_key(__double2float_rd(depth_bound(Mz, Szz, it.t.rad2, cam.F)));
    }
    if (st) {
        atomicOr(it.status, st);
        atomicOr(&B.hdr->status, st);
    }
    keys[it.kern_start + n] = batch_key(key, item, B.item_bits);
    vals[it.kern_start + n] = (uint32_t)n;
}

// One thread per sorted position r: the item comes from the key, the
// kernel's item-local index from the value, its item-local rank is
// r - kern_start.
__global__ __launch_bounds__(PREP_THREADS) void k_prep_records(BatchDev B, int total,
                                                                const uint32_t* __restrict__ skeys,
                                                                const uint32_t* __restrict__ svals,
                                                                CullRec* __restrict__ cull, TraceRec* __restrict__ rec,
                                                                GeoRec* __restrict__ geo) {
    const int r = blockIdx.x * PREP_THREADS + threadIdx.x;
    if (r >= total) return;
    const int ib = B.item_bits;
    const uint32_t key = skeys[r];
    const int item = ib ? (int)(key >> (32 - ib)) : 0;
    const ItemDev& it = B.items[item];
    const uint32_t dmask = ib ? ((1u << (32 - ib)) - 1u) : 0xFFFFFFFFu;
    const bool culled = (key & dmask) == dmask;
    const uint32_t n = svals[r];
    TraceRec tr = {};
    tr.idx = n;
    tr.rank = (uint32_t)(r - it.kern_start);
    tr.tlo = INFINITY;
    CullRec cr;
    cr.i0 = 1; cr.i1 = 0; cr.j0 = 1; cr.j1 = 0;
    cr.tlo = INFINITY;
    cr.pad = 0;
    GeoRec g = {};
    g.idx = n;
    if (!culled) {
        const CamDev& cam = it.cam;
        const double rad2 = it.t.rad2;
        double M0[3], Sig[6], S0[6];
        load_kernel(it.means, it.covs, (int)n, M0, Sig);
        spd_inverse6(Sig, S0);
        double R[9];
        for (int e = 0; e < 9; ++e) R[e] = (double)cam.R[e];
        double M[3];
        for (int d = 0; d < 3; ++d)
            M[d] = R[3 * d] * M0[0] + R[3 * d + 1] * M0[1] + R[3 * d + 2] * M0[2] + (double)cam.T[d];
        double S[6], Sc[6];
        rotate_sym(R, S0, S);       // camera-space inverse covariance
        rotate_sym(R, Sig, Sc);     // camera-space covariance
        const double F = (double)cam.F;
        tr.A0 = S[0];
        tr.A1 = 2.0 * S[1];
        tr.A2 = 2.0 * S[2] * F;
        tr.A3 = S[3];
        tr.A4 = 2.0 * S[4] * F;
        tr.A5 = S[5] * F * F;
        const double w0 = S[0] * M[0] + S[1] * M[1] + S[2] * M[2];
        const double w1 = S[1] * M[0] + S[3] * M[1] + S[4] * M[2];
        const double w2 = S[2] * M[0] + S[4] * M[1] + S[5] * M[2];
        tr.B0 = w0;
        tr.B1 = w1;
        tr.B2 = w2 * F;
        tr.c = M[0] * w0 + M[1] * w1 + M[2] * w2;
        // the bucket's floor: monotone along the sorted order, and no larger
        // than this kernel's own bound
        const float tlo = bucket_floor(key, ib);
        tr.tlo = tlo;
        cr.tlo = tlo;
        for (int d = 0; d < 3; ++d) g.M[d] = M[d];
        for (int e = 0; e < 6; ++e) g.S[e] = S[e];

        // screen bounds of the eta-ellipsoid's silhouette.  With A = 2 ln(1/eta) Sigma_cam
        // and P = M M^T - A, the silhouette's dual conic in (u, v, 1) is
        // diag(F,F,1) P diag(F,F,1); its tangent lines u = const give the row range.
        const double zlo = M[2] - sqrt(rad2 * Sc[5]);
        const int H = cam.H, W = cam.W;
        double i0 = 0.0, i1 = (double)(H - 1), j0 = 0.0, j1 = (double)(W - 1);
        if (zlo > 0.0) {
            const double P00 = M[0] * M[0] - rad2 * Sc[0];
            const double P02 = M[0] * M[2] - rad2 * Sc[2];
            const double P11 = M[1] * M[1] - rad2 * Sc[3];
            const double P12 = M[1] * M[2] - rad2 * Sc[4];
            const double P22 = M[2] * M[2] - rad2 * Sc[5];
            const double du = sqrt(fmax(0.0, P02 * P02 - P00 * P22));
            const double dv = sqrt(fmax(0.0, P12 * P12 - P11 * P22));
            const double margin = 0.01;
            i0 = fmax(i0, floor(F * (P02 - du) / P22 + (double)cam.cy - margin));
            i1 = fmin(i1, ceil(F * (P02 + du) / P22 + (double)cam.cy + margin));
            j0 = fmax(j0, floor(F * (P12 - dv) / P22 + (double)cam.cx - margin));
            j1 = fmin(j1, ceil(F * (P12 + dv) / P22 + (double)cam.cx + margin));
        }
        if (i0 <= i1 && j0 <= j1) {
            cr.i0 = (int16_t)i0; cr.i1 = (int16_t)i1;
            cr.j0 = (int16_t)j0; cr.j1 = (int16_t)j1;
            // coarse stage (binned items): one count per screen tile the box meets
            if (it.t.binned) {
                const int ntx = (W + TILE - 1) / TILE;
                for (int ti = cr.i0 / TILE; ti <= cr.i1 / TILE; ++ti)
                    for (int tj = cr.j0 / TILE; tj <= cr.j1 / TILE; ++tj)
                        atomicAdd(&B.tcnt[it.tile_start + ti * ntx + tj], 1u);
            }
        }
    }
    cull[r] = cr;
    rec[r] = tr;
    geo[r] = g;
}

// ------------------------------------------------------------ block masks
// Which 8x8 blocks of an item's screen some kernel's box meets (select skips
// the others).  A workgroup takes one part of an item's boxes and counts, in
// LDS, the boxes covering each cell of a grid over the image: every box adds
// +1 and -1 at the four corners of its cell range (a difference array), and
// prefix sums along the rows, then down the columns, turn the corner marks
// into the number of boxes over each cell -- four LDS atomics per kernel
// whatever its box's size.  LDS atomics are served about one lane per cycle
// per CU, so an item's boxes are split over up to COVER_SPLIT workgroups of
// COVER_RECS or more boxes, which OR their tiles' bits into the masks
// (cleared by k_prep_keys).  The cells are the 8x8 blocks when their grid
// fits COVER_CELLS, else the 16x16 tiles (a covered tile keeps all four of
// its blocks), else the item is dense (every block scans).
constexpr int COVER_THREADS = 1024;
constexpr int COVER_CELLS = 16384;       // grid cells held in LDS (64 KB)
constexpr int COVER_BATCH = 8;           // boxes per thread loaded together
constexpr int COVER_RECS = 2048;         // boxes per workgroup, at least (but the last part)
constexpr int COVER_SPLIT = 16;          // workgroups per item, at most

// Workgroups per item of a batch whose largest item has max_n kernels.
inline int cover_split(int max_n) {
    return std::max(1, std::min(COVER_SPLIT, (max_n + COVER_RECS - 1) / COVER_RECS));
}

__global__ __launch_bounds__(COVER_THREADS) void k_block_cover(BatchDev B, const CullRec* __restrict__ cull,
                                                               int split) {
    __shared__ int g[COVER_CELLS];
    const int item = blockIdx.x / split, part = blockIdx.x % split;
    const ItemDev& it = B.items[item];
    const int tid = threadIdx.x;
    const int H = it.t.H, W = it.t.W;
    const int nty = (H + TILE - 1) / TILE, ntx = (W + TILE - 1) / TILE;
    // this part's boxes: [r_lo, r_hi) of the item's records
    const int N = it.t.N;
    const int per = std::max(COVER_RECS, (N + split - 1) / split);
    const int r_lo = part * per, r_hi = std::min(N, r_lo + per);
    if (r_lo >= r_hi) return;
    int sh = 3;                              // cell = 2^sh pixels a side
    int nci = (H + 7) >> 3, ncj = (W + 7) >> 3;
    if ((nci + 1) * (ncj + 1) > COVER_CELLS) {
        sh = 4;
        nci = nty;
        ncj = ntx;
    }
    const int gw = ncj + 1, gh = nci + 1;
    if (gh * gw > COVER_CELLS) {
        if (tid == 0) B.tdense[item] = 1u;
        return;
    }
    for (int c = tid; c < gh * gw; c += COVER_THREADS) g[c] = 0;
    __syncthreads();
    // the boxes, COVER_BATCH per thread in flight at a time; every lane loads
    // (past the end: the part's last record, then dropped), so that a
    // batch's loads are all issued before the first wait
    const CullRec* cr = cull + it.kern_start;
    for (int r0 = r_lo + tid; r0 < r_hi; r0 += COVER_BATCH * COVER_THREADS) {
        CullRec b[COVER_BATCH];
#pragma unroll
        for (int u = 0; u < COVER_BATCH; ++u) {
            const int r = r0 + u * COVER_THREADS;
            b[u] = cr[std::min(r, r_hi - 1)];
            if (r >= r_hi) {
                b[u].i0 = 1;
                b[u].i1 = 0;
            }
        }
#pragma unroll
        for (int u = 0; u < COVER_BATCH; ++u) {
            if (b[u].i0 > b[u].i1 || b[u].j0 > b[u].j1) continue;     // culled or past the end: no box
            const int ci0 = b[u].i0 >> sh, ci1 = (b[u].i1 >> sh) + 1;
            const int cj0 = b[u].j0 >> sh, cj1 = (b[u].j1 >> sh) + 1;
            atomicAdd(&g[ci0 * gw + cj0], 1);
            atomicAdd(&g[ci0 * gw + cj1], -1);
            atomicAdd(&g[ci1 * gw + cj0], -1);
            atomicAdd(&g[ci1 * gw + cj1], 1);
        }
    }
    __syncthreads();
    // inclusive prefix sum of the n cells base, base + st, ... by one thread,
    // eight cells loaded together (their loads do not wait for the stores)
    auto scan = [&](int base, int n, int st) {
        int acc = 0;
        for (int c0 = 0; c0 < n; c0 += 8) {
            int v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = c0 + u < n ? g[base + (c0 + u) * st] : 0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                acc += v[u];
                if (c0 + u < n) g[base + (c0 + u) * st] = acc;
            }
        }
    };
    for (int i = tid; i < gh; i += COVER_THREADS) scan(i * gw, gw, 1);
    __syncthreads();
    for (int j = tid; j < gw; j += COVER_THREADS) scan(j, gh, gw);
    __syncthreads();
    for (int t = tid; t < it.t.n_tiles; t += COVER_THREADS) {
        const int ti = t / ntx, tj = t % ntx;
        uint32_t m = 0;
        for (int q = 0; q < 4; ++q) {
            // block (2 ti + q / 2, 2 tj + q % 2); blocks past the image stay clear
            const int ci = (2 * ti + (q >> 1)) >> (sh - 3), cj = (2 * tj + (q & 1)) >> (sh - 3);
            if (ci < nci && cj < ncj && g[ci * gw + cj] > 0) m |= 1u << q;
        }
        if (m) atomicOr(&B.tmask[it.tile_start + t], m);
    }
}

// ------------------------------------------------------- coarse-stage bins
// The tile counts of k_prep_records are scanned into list offsets (blocks of
// TSCAN_BLOCK counts: block sums, one scan of the sums, block scans); then
// every kernel writes its item-local rank into the list of each tile its
// screen box meets.  The order inside a tile's list is whatever the atomics
// give: select sorts a list by rank (= depth order) in LDS before it scans.
// A tile whose list would end past the capacity is not binned (select then
// scans all of its item's records), so a capacity shortfall costs time only.
constexpr int TSCAN_THREADS = 256;
constexpr int TSCAN_PER = TSCAN_BLOCK / TSCAN_THREADS;

__global__ __launch_bounds__(TSCAN_THREADS) void k_tscan_sums(const uint32_t* __restrict__ cnt, int n,
                                                               uint32_t* __restrict__ bsum) {
    __shared__ uint32_t red[TSCAN_THREADS / WAVE];
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * TSCAN_BLOCK + tid * TSCAN_PER;
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < TSCAN_PER; ++j) v += i0 + j < n ? cnt[i0 + j] : 0u;
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (tid % WAVE == 0) red[tid / WAVE] = v;
    __syncthreads();
    if (tid == 0) {
        uint32_t t = 0;
        for (int w = 0; w < TSCAN_THREADS / WAVE; ++w) t += red[w];
        bsum[blockIdx.x] = t;
    }
}

// Block b: the exclusive scan of its counts plus the scanned block sum;
// clears the scatter cursors; the last block writes the grand total at n.
__global__ __launch_bounds__(TSCAN_THREADS) void k_tscan_final(const uint32_t* __restrict__ cnt, int n,
                                                                const uint32_t* __restrict__ bsum, int nblk,
                                                                uint32_t* __restrict__ off, uint32_t* __restrict__ cur) {
    __shared__ uint32_t buf[TSCAN_THREADS];
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * TSCAN_BLOCK + tid * TSCAN_PER;
    uint32_t v[TSCAN_PER];
    uint32_t run = 0;
#pragma unroll
    for (int j = 0; j < TSCAN_PER; ++j) {
        v[j] = i0 + j < n ? cnt[i0 + j] : 0u;
        run += v[j];
    }
    buf[tid] = run;
    __syncthreads();
    for (int o = 1; o < TSCAN_THREADS; o <<= 1) {
        const uint32_t y = tid >= o ? buf[tid - o] : 0u;
        __syncthreads();
        buf[tid] += y;
        __syncthreads();
    }
    uint32_t base = bsum[blockIdx.x] + buf[tid] - run;
#pragma unroll
    for (int j = 0; j < TSCAN_PER; ++j) {
        if (i0 + j < n) {
            off[i0 + j] = base;
            cur[i0 + j] = 0u;
        }
        base += v[j];
    }
    if (blockIdx.x == nblk - 1 && tid == 0) off[n] = bsum[nblk];
}

__global__ __launch_bounds__(PREP_THREADS) void k_bin_scatter(BatchDev B, int total,
                                                               const uint32_t* __restrict__ skeys,
                                                               const CullRec* __restrict__ cull) {
    const int r = blockIdx.x * PREP_THREADS + threadIdx.x;
    if (r >= total) return;
    const int ib = B.item_bits;
    const int item = ib ? (int)(skeys[r] >> (32 - ib)) : 0;
    const ItemDev& it = B.items[item];
    const CullRec cr = cull[r];
    if (!it.t.binned || cr.i0 > cr.i1 || cr.j0 > cr.j1) return;
    const int ntx = (it.t.W + TILE - 1) / TILE;
    const uint32_t rank = (uint32_t)(r - it.kern_start);
    for (int ti = cr.i0 / TILE; ti <= cr.i1 / TILE; ++ti) {
        for (int tj = cr.j0 / TILE; tj <= cr.j1 / TILE; ++tj) {
            const int t = it.tile_start + ti * ntx + tj;
            const uint32_t o = B.toff[t];
            if (o + B.tcnt[t] > B.tcap) continue;          // tile not binned: nothing to write
            const uint32_t pos = atomicAdd(&B.tcur[t], 1u);
            B.tlist[o + pos] = rank;
        }
    }
}

// ------------------------------------------------------------------ sort
// LSD radix sort of (key, value) pairs, 8-bit digits, stable.  A block owns
// SORT_TILE consecutive items; per pass: block histograms (digit-major),
// one exclusive scan, then a stable scatter that ranks equal digits inside a
// wave with ballots and across waves through LDS.
constexpr int SORT_THREADS = 256;
constexpr int SORT_ROUNDS = 2;
constexpr int SORT_TILE = SORT_THREADS * SORT_ROUNDS;

int sort_blocks(int N) { return (N + SORT_TILE - 1) / SORT_TILE; }

__global__ __launch_bounds__(SORT_THREADS) void k_sort_hist(const uint32_t* __restrict__ keys, int N, int shift,
                                                             uint32_t* __restrict__ hist, int nblk) {
    __shared__ uint32_t cnt[256];
    const int tid = threadIdx.x;
    cnt[tid] = 0;
    __syncthreads();
    const int base = blockIdx.x * SORT_TILE;
    for (int it = 0; it < SORT_ROUNDS; ++it) {
        const int i = base + it * SORT_THREADS + tid;
        if (i < N) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(size_t)tid * nblk + blockIdx.x] = cnt[tid];
}

// Per digit d (one workgroup each): exclusive scan of the block counts
// hist[d][0..nblk) in place, and the digit's total in tot[d].
constexpr int SCAN_THREADS = 256;

__global__ __launch_bounds__(SCAN_THREADS) void k_sort_scan(uint32_t* __restrict__ hist, uint32_t* __restrict__ tot,
                                                             int nblk) {
    __shared__ uint32_t buf[SCAN_THREADS];
    const int tid = threadIdx.x;
    uint32_t* h = hist + (size_t)blockIdx.x * nblk;
    uint32_t carry = 0;
    for (int c0 = 0; c0 < nblk; c0 += SCAN_THREADS * 8) {
        // each lane owns 8 consecutive counts of this chunk
        const int b0 = c0 + tid * 8;
        uint32_t v[8];
        uint32_t run = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            v[j] = b0 + j < nblk ? h[b0 + j] : 0u;
            run += v[j];
        }
        buf[tid] = run;
        __syncthreads();
        for (int off = 1; off < SCAN_THREADS; off <<= 1) {
            const uint32_t y = tid >= off ? buf[tid - off] : 0u;
            __syncthreads();
            buf[tid] += y;
            __syncthreads();
        }
        uint32_t base = carry + buf[tid] - run;
        const uint32_t chunk_total = buf[SCAN_THREADS - 1];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (b0 + j < nblk) h[b0 + j] = base;
            base += v[j];
        }
        carry += chunk_total;
        __syncthreads();
    }
    if (tid == 0) tot[blockIdx.x] = carry;
}

__global__ __launch_bounds__(SORT_THREADS) void k_sort_scatter(const uint32_t* __restrict__ kin,
                                                                const uint32_t* __restrict__ vin,
                                                                uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                                int N, int shift, const uint32_t* __restrict__ hist,
                                                                const uint32_t* __restrict__ tot, int nblk) {
    static_assert(SORT_THREADS == 256, "one lane per digit");
    __shared__ uint32_t offs[256];
    __shared__ uint32_t wcnt[SORT_THREADS / WAVE][256];
    const int tid = threadIdx.x, wave = tid / WAVE;
    // digit bases: exclusive scan of the digit totals
    const uint32_t t = tot[tid];
    offs[tid] = t;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t y = tid >= off ? offs[tid - off] : 0u;
        __syncthreads();
        offs[tid] += y;
        __syncthreads();
    }
    const uint32_t dbase = offs[tid] - t;
    __syncthreads();
    offs[tid] = dbase + hist[(size_t)tid * nblk + blockIdx.x];
    const int base = blockIdx.x * SORT_TILE;
    const uint64_t lt = lanemask_lt();
    for (int it = 0; it < SORT_ROUNDS; ++it) {
        const int i = base + it * SORT_THREADS + tid;
        const bool valid = i < N;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t d = (key >> shift) & 255u;
        for (int w = 0; w < SORT_THREADS / WAVE; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = offs[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            kout[pos] = key;
            vout[pos] = vin[i];
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < SORT_THREADS / WAVE; ++w) add += wcnt[w][tid];
        offs[tid] += add;
        __syncthreads();
    }
}

// Small items: one workgroup sorts an item's keys in LDS.  The values are
// the item-local indices, so (key << 32 | index) are distinct and a bitonic
// network over them yields exactly the stable order of the radix sort.
constexpr int ISORT_MAX = 4096;
constexpr int ISORT_THREADS = 1024;

__global__ __launch_bounds__(ISORT_THREADS) void k_sort_items(BatchDev B, uint32_t* __restrict__ keys,
                                                               uint32_t* __restrict__ vals) {
    __shared__ uint64_t s[ISORT_MAX];
    const ItemDev& it = B.items[blockIdx.x];
    const int N = it.t.N, k0 = it.kern_start, tid = threadIdx.x;
    if (N <= 1) return;
    int n2 = 2;
    while (n2 < N) n2 <<= 1;
    for (int i = tid; i < n2; i += ISORT_THREADS)
        s[i] = i < N ? ((uint64_t)keys[k0 + i] << 32) | vals[k0 + i] : ~0ull;
    __syncthreads();
    for (int size = 2; size <= n2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < (n2 >> 1); i += ISORT_THREADS) {
                const int lo = 2 * i - (i & (stride - 1)), hi = lo + stride;
                const uint64_t a = s[lo], b = s[hi];
                const bool ascending = (lo & size) == 0;
                if ((a > b) == ascending) {
                    s[lo] = b;
                    s[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < N; i += ISORT_THREADS) {
        keys[k0 + i] = (uint32_t)(s[i] >> 32);
        vals[k0 + i] = (uint32_t)s[i];
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t n, uint32_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// One block per item: its table record (from the arguments or already in the
// table), its ranges of the block -> item maps, its status word.
__global__ __launch_bounds__(256) void k_init(InitPack P, int first, int from_args, ItemDev* __restrict__ table,
                                              int* __restrict__ tile_item, int* __restrict__ pblk_item,
                                              int* __restrict__ epi_item, WsHeader* __restrict__ hdr,
                                              int clear_status, int clear_header) {
    const int b = blockIdx.x, item = first + b, tid = threadIdx.x;
    if (from_args) {
        static_assert(sizeof(ItemDev) % 4 == 0, "ItemDev is a whole number of words");
        const uint32_t* src = reinterpret_cast<const uint32_t*>(&P.it[b]);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&table[item]);
        for (int w = tid; w < (int)(sizeof(ItemDev) / 4); w += blockDim.x) dst[w] = src[w];
    }
    const ItemDev& it = from_args ? P.it[b] : table[item];
    for (int t = tid; t < it.t.n_tiles; t += blockDim.x) tile_item[it.tile_start + t] = item;
    for (int t = tid; t < it.n_pblk; t += blockDim.x) pblk_item[it.pblk_start + t] = item;
    for (int t = tid; t < it.n_epi; t += blockDim.x) epi_item[it.epi_start + t] = item;
    if (tid == 0 && clear_status) {
        *it.status = 0;
        if (clear_header && b == 0) hdr->status = 0;
    }
}

// ------------------------------------------------------------- launchers
void launch_fill_u32(void* p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return;
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, n, v);
}

void launch_init(const InitPack& pack, int first, int count, bool from_args, ItemDev* table, int* tile_item,
                 int* pblk_item, int* epi_item, WsHeader* hdr, bool clear_status, bool clear_header, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_init, dim3(count), dim3(256), 0, s, pack, first, from_args ? 1 : 0, table, tile_item,
                       pblk_item, epi_item, hdr, clear_status ? 1 : 0, clear_header ? 1 : 0);
}

// The bins of every item's tiles from the records' screen boxes (the counts
// were taken by k_prep_records).
static void launch_bins(const BatchDev& b, int total_kern, int total_tiles, int tscan_blocks, const uint32_t* skeys,
                        uint32_t* tsum, const CullRec* cull, hipStream_t s) {
    if (total_tiles <= 0) return;
    hipLaunchKernelGGL(k_tscan_sums, dim3(tscan_blocks), dim3(TSCAN_THREADS), 0, s, b.tcnt, total_tiles, tsum);
    // the scan of the block sums in place, their total at tsum[tscan_blocks]
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(SCAN_THREADS), 0, s, tsum, tsum + tscan_blocks, tscan_blocks);
    hipLaunchKernelGGL(k_tscan_final, dim3(tscan_blocks), dim3(TSCAN_THREADS), 0, s, b.tcnt, total_tiles, tsum,
                       tscan_blocks, b.toff, b.tcur);
    const int blocks = (total_kern + PREP_THREADS - 1) / PREP_THREADS;
    if (blocks > 0) hipLaunchKernelGGL(k_bin_scatter, dim3(blocks), dim3(PREP_THREADS), 0, s, b, total_kern, skeys, cull);
}

void launch_prep(const BatchDev& b, int total_pblk, int total_kern, int max_n, int total_tiles, int tscan_blocks,
                 uint32_t* keys, uint32_t* vals, uint32_t* keys2, uint32_t* vals2, uint32_t* hist, uint32_t* tsum,
                 CullRec* cull, TraceRec* rec, GeoRec* geo, hipStream_t s) {
    // no binned item: no bins (select reads them only for binned items)
    if (!b.any_binned) total_tiles = 0;
    if (total_tiles > 0) launch_fill_u32(b.tcnt, (size_t)total_tiles, 0u, s);
    if (total_kern <= 0) {
        launch_bins(b, 0, total_tiles, tscan_blocks, keys, tsum, cull, s);
        return;
    }
    hipLaunchKernelGGL(k_prep_keys, dim3(total_pblk), dim3(PREP_THREADS), 0, s, b, keys, vals);
    const int N = total_kern;
    const int blocks = (N + PREP_THREADS - 1) / PREP_THREADS;
    if (max_n <= ISORT_MAX) {
        // every item sorts in one workgroup's LDS
        hipLaunchKernelGGL(k_sort_items, dim3(b.n_items), dim3(ISORT_THREADS), 0, s, b, keys, vals);
        hipLaunchKernelGGL(k_prep_records, dim3(blocks), dim3(PREP_THREADS), 0, s, b, N, keys, vals, cull, rec, geo);
        if (b.masks)
            hipLaunchKernelGGL(k_block_cover, dim3(b.n_items * cover_split(max_n)), dim3(COVER_THREADS), 0, s, b,
                               cull, cover_split(max_n));
        launch_bins(b, N, total_tiles, tscan_blocks, keys, tsum, cull, s);
        return;
    }
    // four stable 8-bit passes: keys/vals -> keys2/vals2 -> keys/vals -> ...
    const int nblk = sort_blocks(N);
    uint32_t* kin = keys;
    uint32_t* vin = vals;
    uint32_t* kout = keys2;
    uint32_t* vout = vals2;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_sort_hist, dim3(nblk), dim3(SORT_THREADS), 0, s, kin, N, shift, hist, nblk);
        hipLaunchKernelGGL(k_sort_scan, dim3(256), dim3(SCAN_THREADS), 0, s, hist, hist + (size_t)256 * nblk,
                           nblk);
        hipLaunchKernelGGL(k_sort_scatter, dim3(nblk), dim3(SORT_THREADS), 0, s, kin, vin, kout, vout, N, shift,
                           hist, hist + (size_t)256 * nblk, nblk);
        uint32_t* t = kin; kin = kout; kout = t;
        t = vin; vin = vout; vout = t;
    }
    hipLaunchKernelGGL(k_prep_records, dim3(blocks), dim3(PREP_THREADS), 0, s, b, N, kin, vin, cull, rec, geo);
    if (b.masks)
        hipLaunchKernelGGL(k_block_cover, dim3(b.n_items * cover_split(max_n)), dim3(COVER_THREADS), 0, s, b, cull,
                           cover_split(max_n));
    launch_bins(b, N, total_tiles, tscan_blocks, kin, tsum, cull, s);
}

}  // namespace voge
