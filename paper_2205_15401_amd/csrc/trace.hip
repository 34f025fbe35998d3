// trace.hip -- per-pixel ray tracing and K-nearest selection (k_select),
// erf-sum transmittance and blending (k_blend), and the backward (k_bwd).
//
// Every kernel maps one workgroup of 256 lanes to one 16x16 screen tile of
// some item of the batch; each wave owns an 8x8 block and each lane one
// pixel.  Per-pixel kept lists travel between the kernels through the
// workspace, slot-major per item: list[s * S + q] with q = tile * 256 +
// lane-in-tile and S = n_tiles * 256, so every list access of a wave is one
// contiguous segment.
//
//   k_select -- coarse stage + ray tracing + fine selection.  Each wave
//     scans its item's depth-ordered records 64 at a time, keeps those whose
//     screen box meets its block, and every pixel traces them in order
//     (VoGE Sec. 3.3, Eq. 6; App. A.1) along D' = (i - O_y, j - O_x, F):
//         a = D'^T S D',  b = D'^T S M,  l = b / a,  -2q = M^T S M - b l   (FP64)
//     and keeps e^q > eta, l > 0, the K smallest l (Sec. 3.3; App. A.3).
//     A candidate is a 64-bit key: the bits of l (a positive double) with the
//     low 24 bits replaced by the kernel's rank, so one unsigned compare
//     orders by (l, rank); the K-buffer holds the kept keys in registers, in
//     no order (a full buffer's largest key is the one a nearer key replaces).
//     A pixel is done once its K-th entry is nearer than the next record's
//     depth floor; the wave stops when all its pixels are done.
//   k_blend -- E_k = sum_m e^{q_m} Phi((l_k - l_m) sqrt(a_m)) (Eq. 7 at
//     t = l_k; App. A.2), T_k = exp(-E_k), W_k = T_k e^{q_k}, C = sum W_k c_k (Eq. 8).
//   k_bwd -- gradients of C with the kept sets fixed (formulas above
//     bwd_pix_body): a pixel phase, then a tile reduction.
//
// D' is F times the paper's D: l * D', q, the erf arguments and every weight
// are unchanged by that scale; only l itself scales.
#include "voge_internal.hpp"
#include "voge_launch.hpp"

namespace voge {

constexpr float INV_SQRT_PI = 0.564189583547756287f;

// Phi(x) = (1 + erf x)/2 = erfc(-x)/2, with erfc(z), z = |x|, as
//   erfc(z) = t Q(t) e^{-z^2},   t = 1/(1 + z/2),
// Q a degree-8 polynomial fitted to e^{z^2} erfc(z) / t (relative error
// 4.5e-8; the fit and its method: phi_fit.py; the coefficients below are
// Q's halved).  The argument comes scaled, xs = x sqrt(log2 e), so that
// e^{-x^2} = 2^{-xs^2} is one multiply and one hardware exp2; then
// t = 1/(1 + z/2) = 1/(1 + |xs| / (2 sqrt(log2 e))).  In FP32,
// |Phi - (1 + erf x)/2| < 2e-7.  Branch-free: one reciprocal and the
// exponential, which the backward shares with the density
// Phi'(x) = e^{-x^2}/sqrt(pi).
constexpr float SQRT_LOG2E = 1.20112240878645f;       // sqrt(log2 e)
constexpr float HALF_OVER_SQRT_LOG2E = 0.416277306f;  // 1 / (2 sqrt(log2 e))

// e^{-x^2} from the scaled argument xs = x sqrt(log2 e)
__device__ __forceinline__ float gauss_scaled(float xs) { return __builtin_amdgcn_exp2f(-xs * xs); }

__device__ __forceinline__ float phi_from(float xs, float e) {
    const float z = fabsf(xs);
    const float t = __builtin_amdgcn_rcpf(fmaf(HALF_OVER_SQRT_LOG2E, z, 1.0f));
    float q = fmaf(t, -0.0297155753f, 0.143165097f);
    q = fmaf(t, q, -0.245402336f);
    q = fmaf(t, q, 0.141075402f);
    q = fmaf(t, q, -0.0147031052f);
    q = fmaf(t, q, 0.101923697f);
    q = fmaf(t, q, 0.121407524f);
    q = fmaf(t, q, 0.141207144f);
    q = fmaf(t, q, 0.141042113f);
    const float h = t * q * e;                     // erfc(z) / 2
    return xs >= 0.f ? 1.0f - h : h;
}

__device__ __forceinline__ float phi_cdf(float x) {
    const float xs = x * SQRT_LOG2E;
    return phi_from(xs, gauss_scaled(xs));
}

struct PixelCtx {
    int pi, pj;
    bool valid;
    double u, v;
    size_t q;     // list index
};

// Pixel `slot` (0..255) of a tile: slot s sits in the 8x8 block s / 64 at
// row (s % 64) / 8, column s % 8 of that block; its lists live at
// tile * 256 + s.
__device__ __forceinline__ PixelCtx pixel_at(int tile, int slot, int ntx, int H, int W, float cx, float cy) {
    const int blk = slot / WAVE, within = slot % WAVE;
    const int ti0 = (tile / ntx) * TILE, tj0 = (tile % ntx) * TILE;
    PixelCtx P;
    P.pi = ti0 + (blk >> 1) * 8 + (within >> 3);
    P.pj = tj0 + (blk & 1) * 8 + (within & 7);
    P.valid = P.pi < H && P.pj < W;
    P.u = (double)P.pi - (double)cy;
    P.v = (double)P.pj - (double)cx;
    P.q = (size_t)tile * TILE_THREADS + slot;
    return P;
}

// The lane's own pixel: slot = lane id in the workgroup.
__device__ __forceinline__ PixelCtx pixel_of(int tile, int ntx, int H, int W, float cx, float cy) {
    return pixel_at(tile, threadIdx.x, ntx, H, W, cx, cy);
}

// The tile's pixels regrouped by kept count (largest first), so that each
// wave's pixels have similar counts: the per-pixel pair loops run to the
// wave's largest count.  Returns the slot this lane works on.  Which lane
// computes which pixel does not change any result.
__device__ __forceinline__ int balanced_slot(const TraceArgs& A, int tile, int ntx) {
    __shared__ int s_bin[MAX_K + 2];
    __shared__ int s_perm[TILE_THREADS];
    const int tid = threadIdx.x;
    const PixelCtx P = pixel_of(tile, ntx, A.H, A.W, A.cx, A.cy);
    const int ke = P.valid ? gp(A.keff)[P.q] : 0;
    const int bin = MAX_K - ke;                  // descending counts
    if (tid < MAX_K + 2) s_bin[tid] = 0;
    __syncthreads();
    const int pos = atomicAdd(&s_bin[bin], 1);
    __syncthreads();
    if (tid < WAVE) {
        // exclusive scan of the MAX_K + 1 bins by the first wave (two per lane)
        const int b0 = 2 * tid, b1 = 2 * tid + 1;
        const int c0 = b0 <= MAX_K ? s_bin[b0] : 0, c1 = b1 <= MAX_K ? s_bin[b1] : 0;
        int run = c0 + c1;
        for (int off = 1; off < WAVE; off <<= 1) {
            const int y = __shfl_up(run, off);
            if (tid >= off) run += y;
        }
        const int ex = run - c0 - c1;
        if (b0 <= MAX_K) s_bin[b0] = ex;
        if (b1 <= MAX_K) s_bin[b1] = ex + c0;
    }
    __syncthreads();
    s_perm[s_bin[bin] + pos] = tid;
    __syncthreads();
    return s_perm[tid];
}

// 1 / a for a > 0: hardware reciprocal estimate and two Newton steps.
__device__ __forceinline__ double rcp_pos(double a) {
    double r = __builtin_amdgcn_rcp(a);
    r = fma(fma(-a, r, 1.0), r, r);
    return fma(fma(-a, r, 1.0), r, r);
}

// b / a for a > 0: hardware reciprocal estimate, two Newton steps and a
// residual correction (within an ulp or two of the rounded quotient).
__device__ __forceinline__ double div_pos(double b, double a) {
    double r = __builtin_amdgcn_rcp(a);
    r = fma(fma(-a, r, 1.0), r, r);
    r = fma(fma(-a, r, 1.0), r, r);
    const double q = b * r;
    return fma(fma(-a, q, b), r, q);
}

// The ray-tracing formulas; explicit fma() fixes the evaluation order so
// every recomputation reproduces the same bits.
template <typename Rec>
__device__ __forceinline__ void trace_one(const Rec& R, double u, double v, double& l, double& q2, double& a) {
    a = fma(u, fma(R.A0, u, fma(R.A1, v, R.A2)), fma(v, fma(R.A3, v, R.A4), R.A5));
    const double b = fma(R.B0, u, fma(R.B1, v, R.B2));
    l = div_pos(b, a);
    q2 = fma(-b, l, R.c);
}

// The trace records as constant memory: the records do not change while
// the trace kernels run, and a uniform index into this address space is
// read with scalar loads into scalar registers.
typedef const __attribute__((address_space(4))) TraceRec* ConstRecPtr;

__device__ __forceinline__ ConstRecPtr const_rec(const TraceRec* p) {
    return (ConstRecPtr)(uintptr_t)p;
}

// The fields the trace needs, read through the constant-space pointer.
__device__ __forceinline__ TraceRec load_rec(ConstRecPtr p) {
    TraceRec r;
    r.A0 = p->A0; r.A1 = p->A1; r.A2 = p->A2; r.A3 = p->A3; r.A4 = p->A4; r.A5 = p->A5;
    r.B0 = p->B0; r.B1 = p->B1; r.B2 = p->B2; r.c = p->c;
    r.tlo = p->tlo;
    r.idx = 0; r.rank = 0; r.pad = 0;
    return r;
}

__device__ __forceinline__ double key_upper_l(uint64_t key) {
    return __longlong_as_double((long long)(key | RANK_MASK));
}

// The K-buffer of a pixel: its kept keys in slots 0 .. n-1, in no order
// (what uses the kept set -- the transmittance sums, the blend and the
// backward -- does not depend on the order).  Slot loops run over groups of
// four under wave-uniform branches up to a uniform bound of the fill counts.

// Write key nk into slot t (t = -1: this lane inserts nothing): a lane
// holding n < K keys appends at t = n, a full lane overwrites the slot of its
// largest key.  One in-place pass over the groups of four slots up to lim
// (lim wave-uniform: the largest fill count, or K-1 when a full lane
// inserts) that some lane writes, one compare and two selects per slot.
template <int KB>
__device__ __forceinline__ void kbuf_put(uint64_t (&key)[KB], uint64_t nk, int t, int lim) {
    const int tg = t >> 2;                       // the lane's group of four slots (-1: none)
#pragma unroll
    for (int s0 = 0; s0 < KB; s0 += 4) {
        // only groups that some lane writes (a vote per group: the writes of
        // one candidate land in one or two groups, appends near the fill counts)
        if (s0 <= lim && wave_any(tg == (s0 >> 2))) {
#pragma unroll
            for (int s = s0; s < s0 + 4 && s < KB; ++s) key[s] = s == t ? nk : key[s];
        }
    }
}

// The largest of the K keys in slots 0 .. K-1 (a full buffer) and its slot.
template <int KB>
__device__ __forceinline__ void kbuf_max(const uint64_t (&key)[KB], int K, uint64_t& mx, int& ms) {
    mx = 0;
    ms = 0;
#pragma unroll
    for (int s0 = 0; s0 < KB; s0 += 4) {
        if (s0 < K) {
#pragma unroll
            for (int s = s0; s < s0 + 4 && s < KB; ++s) {
                const bool gt = s < K && key[s] > mx;
                mx = gt ? key[s] : mx;
                ms = gt ? s : ms;
            }
        }
    }
}

// Block -> tile.  Workgroups are dealt round-robin to the 8 XCDs (block b
// runs on XCD b % 8).  Order 0 (banded): each XCD renders a contiguous band
// of tiles, so the kernels those tiles share stay in that XCD's L2.  Order 1
// (plain): block b renders tile b, so every XCD takes every eighth tile.
__device__ __forceinline__ int tile_of_block(int order) {
    const int b = blockIdx.x, nb = gridDim.x;
    if (order == 1) return b;
    const int x = b & 7, local = b >> 3;
    const int per = nb >> 3, rem = nb & 7;
    return x * per + (x < rem ? x : rem) + local;
}

// Largest kept count in the wave, as a scalar (uniform branches on it).
__device__ __forceinline__ int wave_max_keff(int keff) {
    int kmax = keff;
    for (int off = WAVE / 2; off > 0; off >>= 1) kmax = max(kmax, __shfl_xor(kmax, off));
    return __builtin_amdgcn_readfirstlane(kmax);
}

// ------------------------------------------------------------------ select
// Each wave owns one 8x8 block of the tile and works alone (no workgroup
// barriers: waves with fewer candidates do not wait for the others).  It
// scans the depth-ordered cull records 64 at a time; the records whose
// screen box meets its block are the set bits of a ballot, taken in record
// order with scalar bit scans, and traced one after the other.  Their trace
// records come through the scalar cache, the next candidate's while the
// current one is inserted; nothing in the candidate loop touches LDS, so
// waiting for the current record never waits for anything else.  Per-lane
// decisions stay lane masks, combined with bitwise operators and wave votes
// on the masks rather than branches: the loop is bound by instruction issue,
// and exec-mask bookkeeping had cost as many scalar instructions as the
// trace's vector ones.
// Cull steps loaded ahead in select (one at the deepest K-buffer, whose
// registers are all taken by the keys).
__host__ __device__ constexpr int cull_ahead(int KB) { return KB >= 64 ? 1 : 3; }

// Longest tile list select sorts in LDS (a longer one is scanned unbinned).
constexpr int BIN_MAX = 2048;

// The tile's bin, sorted by rank (= depth order) into s_rank[0 .. n); returns
// n, or -1 when the tile is not binned (its item is not, or its list is
// longer than BIN_MAX or did not fit the pair list).  Every lane of the
// workgroup calls it.
__device__ __forceinline__ int load_bin(const TraceArgs& A, int tile, uint32_t* s_rank) {
    const int tid = threadIdx.x;
    if (!A.binned) return -1;
    const uint32_t cnt = A.tcnt[tile], off = A.toff[tile];
    if (cnt > (uint32_t)BIN_MAX || off + cnt > A.tcap) return -1;
    const int n = (int)cnt;
    int n2 = 2;
    while (n2 < n) n2 <<= 1;
    const auto src = gp(A.tlist) + off;
    for (int i = tid; i < n2; i += TILE_THREADS) s_rank[i] = i < n ? src[i] : 0xFFFFFFFFu;
    __syncthreads();
    // bitonic sort, ascending (ranks are distinct; padding sorts last)
    for (int size = 2; size <= n2 && n > 1; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < (n2 >> 1); i += TILE_THREADS) {
                const int lo = 2 * i - (i & (stride - 1)), hi = lo + stride;
                const uint32_t a = s_rank[lo], b = s_rank[hi];
                if ((a > b) == ((lo & size) == 0)) {
                    s_rank[lo] = b;
                    s_rank[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    return n;
}

// BIN: the candidate stream is the tile's bin, n_list ranks in depth order
// in s_rank (LDS); otherwise it is every record of the item (n_list = N),
// entry j being rank j.
template <int KB, bool BIN>
__device__ __forceinline__ void select_body(const TraceArgs& A, int tile, int blk, const uint32_t* s_rank,
                                            const int n_list) {
    constexpr int CULL_AHEAD = cull_ahead(KB);
    const int lane = threadIdx.x % WAVE;
    const int wave = blk;                        // the tile's 8x8 block of this wave (uniform)
    const int ntx = (A.W + TILE - 1) / TILE;
    const PixelCtx P = pixel_at(tile, wave * WAVE + lane, ntx, A.H, A.W, A.cx, A.cy);
    const int bi0 = (tile / ntx) * TILE + (wave >> 1) * 8;            // this wave's block
    const int bj0 = (tile % ntx) * TILE + (wave & 1) * 8;
    const ConstRecPtr crec = const_rec(A.rec);
    // entry j of the stream: its rank
    auto rank_of = [&](int pos) -> int {
        if constexpr (BIN)
            return (int)s_rank[pos];
        else
            return pos;
    };

    uint64_t key[KB];
#pragma unroll
    for (int s = 0; s < KB; ++s) key[s] = ~0ull;
    uint64_t kth = ~0ull;                        // the largest kept key once K are kept
    int nkey = 0;                                // kept keys (at most K)
    int ub = 0;                                  // the wave's largest nkey (uniform)
    int kslot = 0;                               // the slot of kth
    // a block that no kernel's screen box meets has no candidate: it keeps
    // nothing and scans nothing
    const bool empty = gp(A.tdense)[0] == 0u && ((gp(A.tmask)[tile] >> wave) & 1u) == 0u;
    bool done = !P.valid || empty;
    // One step: the list entries base .. base+63 (lane j holds the rank of
    // entry base + j in ent) whose boxes meet the block (hit); returns true
    // once the block is done.
    auto step = [&](const int base, const bool hit, const int ent) -> bool {
        uint64_t mm = wave_ballot(hit);          // this step's candidates, one bit per entry
        if (mm != 0) {
            int rank = BIN ? __builtin_amdgcn_readlane(ent, (int)__builtin_ctzll(mm)) : base + (int)__builtin_ctzll(mm);
            mm &= mm - 1;
            TraceRec R = load_rec(crec + rank);
            for (;;) {
                // a lane's early exit needs a full buffer (ub < K: none is, and
                // done has kept its initial value)
                if (ub >= A.K) {
                    if (wave_all(done)) break;
                    done = done | ((kth != ~0ull) & ((double)R.tlo > key_upper_l(kth)));
                }
                // every lane traces (a branch around the trace would cost more
                // than the finished lanes' share of it)
                double l, q2, a;
                trace_one(R, P.u, P.v, l, q2, a);
                const uint64_t nk = ((uint64_t)__double_as_longlong(l) & ~RANK_MASK) | (uint64_t)rank;
                const bool ins = !done & (q2 < A.rad2) & (l > 0.0) & (nk < kth);
                // the next candidate's record is in flight while this one is inserted
                const bool more = mm != 0;
                const int nxt = (int)__builtin_ctzll(mm);
                const int rank_n = !more ? rank : BIN ? __builtin_amdgcn_readlane(ent, nxt) : base + nxt;
                mm &= mm - 1;
                __builtin_amdgcn_sched_barrier(0);
                const TraceRec Rn = load_rec(crec + rank_n);
                if (wave_any(ins)) {
                    // the wave's largest fill count grows by one when a lane at it appends
                    const bool grow = wave_any(ins & (nkey == ub) & (nkey < A.K));
                    const int lim = wave_any(ins & (nkey >= A.K)) ? A.K - 1 : ub;
                    kbuf_put<KB>(key, nk, !ins ? -1 : nkey < A.K ? nkey : kslot, lim);
                    nkey += (ins & (nkey < A.K)) ? 1 : 0;
                    // the largest key (and its slot) of every lane that is full now
                    if (wave_any(ins & (nkey >= A.K))) {
                        uint64_t mx;
                        int ms;
                        kbuf_max<KB>(key, A.K, mx, ms);
                        const bool full = ins & (nkey >= A.K);
                        kth = full ? mx : kth;
                        kslot = full ? ms : kslot;
                    }
                    ub += grow ? 1 : 0;
                }
                if (!more) break;
                R = Rn;
                rank = rank_n;
            }
        }
        // the block is done when every pixel is, or holds K kernels nearer
        // than the next entry's depth bound (possible once a buffer is full)
        const int nb = base + WAVE;
        bool fin = done;
        if (ub >= A.K && nb < n_list) {
            // (a readfirstlane of the record scan's uniform position makes the
            // compiler treat the scan position as divergent: records would then
            // come through vector loads into 30-odd more VGPRs)
            int nbr = nb;
            if constexpr (BIN) nbr = __builtin_amdgcn_readfirstlane(rank_of(nb));
            const float next_tlo = crec[nbr].tlo;
            fin = fin | ((kth != ~0ull) & ((double)next_tlo > key_upper_l(kth)));
        }
        return wave_all(fin);
    };

    // The screen boxes of the next CULL_AHEAD steps are in flight (a step
    // with no candidate is a few instructions, far shorter than a load).  The
    // loop is unrolled by CULL_AHEAD so that each box keeps its registers and
    // is reloaded right after its use, and every lane loads (lanes past the
    // last record reload that record, and r < N rejects them), so that
    // waiting for the oldest load leaves the younger ones in flight.
    // (entries past the end reload the last one, and r < n_list rejects them)
    const int n_scan = wave_all(done) ? 0 : n_list;   // a block wholly outside the image scans nothing
    const int last = n_list - 1;
    const auto cull = gp(A.cull);
    auto entry = [&](int pos) -> int { return rank_of(min(pos, last)); };
    CullBox ahead[CULL_AHEAD];
    int ahead_e[BIN ? CULL_AHEAD : 1];          // the entries' ranks (a bin's only)
    if (n_scan > 0) {
#pragma unroll
        for (int d = 0; d < CULL_AHEAD; ++d) {
            if constexpr (BIN) {
                ahead_e[d] = entry(lane + d * WAVE);
                ahead[d] = load_box(cull + ahead_e[d]);
            } else {
                ahead[d] = load_box(cull + entry(lane + d * WAVE));
            }
        }
    }
    bool stop = n_scan == 0;
    for (int base0 = 0; !stop; base0 += CULL_AHEAD * WAVE) {
#pragma unroll
        for (int d = 0; d < CULL_AHEAD; ++d) {
            const int base = base0 + d * WAVE, r = base + lane;
            const CullBox c = ahead[d];
            int e = 0;
            if constexpr (BIN) {
                e = ahead_e[d];
                ahead_e[d] = entry(r + CULL_AHEAD * WAVE);
                ahead[d] = load_box(cull + ahead_e[d]);   // on every path
            } else {
                ahead[d] = load_box(cull + entry(r + CULL_AHEAD * WAVE));
            }
            if (!stop && base < n_scan) {
                const bool hit = (r < n_list) & (c.i0 <= bi0 + 7) & (c.i1 >= bi0) & (c.j0 <= bj0 + 7) & (c.j1 >= bj0);
                stop = step(base, hit, e);
            } else {
                stop = true;
            }
        }
    }

    // write the kept list: FP64 depth, e^q, sqrt(a), rank, original index.
    // Slots below the wave's largest fill count: every lane loads a record
    // (a lane without the slot loads record 0 and discards it), so that a
    // slot's loads are issued together and waited for once.
    const size_t S = A.S;
    const auto rec = gp(A.rec);
#pragma unroll
    for (int s = 0; s < KB; ++s) {
        if (s < ub) {
            const bool has = key[s] != ~0ull;
            const int rank = has ? (int)(key[s] & RANK_MASK) : 0;
            const auto Rp = rec + rank;
            TraceRec R;
            R.A0 = Rp->A0; R.A1 = Rp->A1; R.A2 = Rp->A2; R.A3 = Rp->A3; R.A4 = Rp->A4; R.A5 = Rp->A5;
            R.B0 = Rp->B0; R.B1 = Rp->B1; R.B2 = Rp->B2; R.c = Rp->c;
            R.idx = Rp->idx;
            double l, q2, a;
            trace_one(R, P.u, P.v, l, q2, a);
            if (has) {
                const size_t o = (size_t)s * S + P.q;
                gp(A.kl_l)[o] = l;
                gp(A.kl_m)[o] = expf(-0.5f * (float)q2);
                gp(A.kl_s)[o] = (float)sqrt(a);
                gp(A.kl_r)[o] = rank;
                gp(A.kl_i)[o] = (int)R.idx;
            }
        }
    }
    gp(A.keff)[P.q] = nkey;
}

// ----------------------------------------------------------------- sampler
//
// The sampler of Sec. 3.4 (Eq. 10) rides on the blend: once the blend has
// written a pixel's transmittances, the lane adds W_k = T_k e^{q_k} and
// W_k phi_p to its kernels' entries in a per-tile table in LDS (a hash on the
// original kernel index, float atomic adds); after a barrier each used entry
// makes one global atomic add per value.  Feature maps of more than SAMPLE_CH channels take
// one pass per SAMPLE_CH channels over the same table; pairs whose kernel
// finds the table full go to global memory directly.
constexpr int SAMPLE_HCAP = 1024;     // distinct kernels per tile held in LDS
constexpr int SAMPLE_CH = 8;          // feature channels per pass

size_t sample_lds_bytes(int max_c) {
    const int nv = (max_c < SAMPLE_CH ? max_c : SAMPLE_CH) + 1;
    return (size_t)SAMPLE_HCAP * (1 + nv) * sizeof(float);
}

__device__ __forceinline__ int hash_insert(int* s_key, int hmask, int key) {
    int h = (int)(((uint32_t)key * 2654435761u) >> 7) & hmask;
    for (int probe = 0; probe <= hmask; ++probe) {
        const int cur = atomicCAS(&s_key[h], -1, key);
        if (cur == -1 || cur == key) return h;
        h = (h + 1) & hmask;
    }
    return -1;
}

// `q`: the pixel's list index; its weights are read back from the lists the
// blend has just written (W = T e^q, the product the blend forms).
__device__ __forceinline__ void sample_tile(const TraceArgs& A, bool valid, size_t q, size_t p, int keff,
                                            unsigned char* smem) {
    const int tid = threadIdx.x;
    const int C = A.C;
    const size_t S = A.S;
    const int nv = min(C, SAMPLE_CH) + 1;        // per entry: the weight sum, then one pass's channels
    int* s_key = reinterpret_cast<int*>(smem);
    float* s_val = reinterpret_cast<float*>(s_key + SAMPLE_HCAP);
    for (int i = tid; i < SAMPLE_HCAP; i += TILE_THREADS) s_key[i] = -1;
    for (int i = tid; i < SAMPLE_HCAP * nv; i += TILE_THREADS) s_val[i] = 0.f;
    __syncthreads();
    const auto phi = gp(A.grad_image) + p * C;
    const auto pT = gp(A.kl_T) + q;
    const auto pm = gp(A.kl_m) + q;
    const auto pi = gp(A.kl_i) + q;
    for (int c0 = 0; c0 == 0 || c0 < C; c0 += SAMPLE_CH) {
        const int nc = min(SAMPLE_CH, C - c0);
        if (c0 > 0) {
            for (int i = tid; i < SAMPLE_HCAP * nv; i += TILE_THREADS) s_val[i] = 0.f;
            __syncthreads();
        }
        float f[SAMPLE_CH];
#pragma unroll
        for (int c = 0; c < SAMPLE_CH; ++c) f[c] = (valid && keff > 0 && c < nc) ? phi[c0 + c] : 0.f;
        // slot k+1 is loaded while slot k is added
        float Tn = keff > 0 ? pT[0] : 0.f, mn = keff > 0 ? pm[0] : 0.f;
        int in = keff > 0 ? pi[0] : 0;
        for (int k = 0; k < keff; ++k) {
            const float w = Tn * mn;
            const int key = in;
            if (k + 1 < keff) {
                const size_t o = (size_t)(k + 1) * S;
                Tn = pT[o];
                mn = pm[o];
                in = pi[o];
            }
            // the kernel's entry (inserted by the first pass, found by later ones)
            const int h = hash_insert(s_key, SAMPLE_HCAP - 1, key);
            if (h >= 0) {
                float* v = s_val + h * nv;
                if (c0 == 0) atomicAdd(v, w);
#pragma unroll
                for (int c = 0; c < SAMPLE_CH; ++c)
                    if (c < nc) atomicAdd(v + 1 + c, w * f[c]);
            } else {
                if (c0 == 0) global_add(&A.gW[key], w);
#pragma unroll
                for (int c = 0; c < SAMPLE_CH; ++c)
                    if (c < nc) global_add(&A.gA[(size_t)key * C + c0 + c], w * f[c]);
            }
        }
        __syncthreads();
        for (int i = tid; i < SAMPLE_HCAP; i += TILE_THREADS) {
            const int key = s_key[i];
            if (key < 0) continue;
            const float* v = s_val + i * nv;
            if (c0 == 0) global_add(&A.gW[key], v[0]);
            for (int c = 0; c < nc; ++c) global_add(&A.gA[(size_t)key * C + c0 + c], v[1 + c]);
        }
        if (c0 + SAMPLE_CH < C) __syncthreads();
    }
}

// ------------------------------------------------------------------- blend
// The blend's sums E_k = sum_m e^{q_m} Phi((l_k - l_m) sqrt(a_m)) of the
// pixel at list index q (keff kept kernels; kmax the wave's largest count):
// its kept depths into lk (0 past keff), the sums into E.  m streams from the
// list (slot m+1 is loaded while slot m is computed), k sits in registers.
// List loads are made by every lane of the wave, from slots below the
// wave's largest kept count (which every lane's list has room for), and
// lanes past their own count discard the value: loads under per-lane
// branches would make the compiler wait for every load at once, the one
// issued ahead included.
template <int KB>
__device__ __forceinline__ void blend_sums(const TraceArgs& A, size_t q, int keff, int kmax, double (&lk)[KB],
                                           float (&E)[KB]) {
    const size_t S = A.S;
    const auto pl = gp(A.kl_l) + q;
    const auto pm = gp(A.kl_m) + q;
    const auto ps = gp(A.kl_s) + q;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        lk[k] = 0.0;
        E[k] = 0.f;
        if (k < kmax) {
            const double v = pl[(size_t)k * S];
            lk[k] = k < keff ? v : 0.0;
        }
    }
    double ln = 0.0;
    float mn = 0.f, sn = 1.f;
    if (kmax > 0) {
        const double a = pl[0];
        const float b = pm[0], c = ps[0];
        ln = keff > 0 ? a : 0.0;
        mn = keff > 0 ? b : 0.f;
        sn = keff > 0 ? c : 1.f;
    }
    for (int m = 0; m < kmax; ++m) {
        const double lm = ln;
        const float mm = mn, sms = sn * SQRT_LOG2E;
        const bool nin = m + 1 < keff;
        const size_t o = (size_t)(m + 1 < kmax ? m + 1 : m) * S;
        const double a = pl[o];
        const float b = pm[o], c = ps[o];
        ln = nin ? a : 0.0;
        mn = nin ? b : 0.f;
        sn = nin ? c : 1.f;
        // four independent pairs per uniform branch, so their chains interleave
#pragma unroll
        for (int k0 = 0; k0 < KB; k0 += 4) {
            if (k0 < kmax) {
#pragma unroll
                for (int k = k0; k < k0 + 4 && k < KB; ++k) {
                    const float xs = (float)(lk[k] - lm) * sms;
                    E[k] = fmaf(mm, phi_from(xs, gauss_scaled(xs)), E[k]);
                }
            }
        }
    }
}

// The kept original indices of the pixel at list index q, written to the
// image's kept array in ascending depth (the list itself is unordered):
// slot k goes to the number of kept kernels nearer than it (equal depths in
// slot order).
__device__ __forceinline__ void write_kept(const TraceArgs& A, size_t q, size_t p, int keff) {
    const size_t S = A.S;
    const auto pl = gp(A.kl_l) + q;
    const auto kp = gp(A.kept) + p * A.K;
    for (int s = keff; s < A.K; ++s) kp[s] = -1;
    for (int k = 0; k < keff; ++k) {
        const double l = pl[(size_t)k * S];
        int pos = 0;
        for (int m = 0; m < keff; ++m) {
            const double lm = pl[(size_t)m * S];
            pos += (lm < l || (lm == l && m < k)) ? 1 : 0;
        }
        kp[pos] = gp(A.kl_i)[(size_t)k * S + q];
    }
}

// SAMPLE: also run the sampler on the tile (smem: sample_lds_bytes).
template <int KB, bool SAMPLE>
__device__ __forceinline__ void blend_body(const TraceArgs& A, int tile, unsigned char* smem) {
    const int ntx = (A.W + TILE - 1) / TILE;
    const PixelCtx P = pixel_at(tile, balanced_slot(A, tile, ntx), ntx, A.H, A.W, A.cx, A.cy);
    const size_t S = A.S;
    const int keff = P.valid ? gp(A.keff)[P.q] : 0;
    const int kmax = wave_max_keff(keff);
    const auto pm = gp(A.kl_m) + P.q;
    double lk[KB];
    float E[KB];
    blend_sums<KB>(A, P.q, keff, kmax, lk, E);
    if (!SAMPLE && !P.valid) return;
    const size_t p = (size_t)P.pi * A.W + P.pj;
    float Wt[KB];
    int ik[KB];
    float ws = 0.f;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        Wt[k] = 0.f;
        ik[k] = 0;
    }
#pragma unroll
    for (int k0 = 0; k0 < KB; k0 += 4) {
        if (k0 < kmax) {
            // e^{q_k} and the original indices of four slots, loaded together
            float mq[4];
            int iq[4];
#pragma unroll
            for (int k = k0; k < k0 + 4; ++k) {
                const size_t o = (size_t)(k < kmax ? k : kmax - 1) * S;
                mq[k - k0] = pm[o];
                iq[k - k0] = gp(A.kl_i)[o + P.q];
            }
#pragma unroll
            for (int k = k0; k < k0 + 4; ++k) {
                const float T = expf(-E[k]);
                if (k < keff) gp(A.kl_T)[(size_t)k * S + P.q] = T;
                Wt[k] = k < keff ? T * mq[k - k0] : 0.f;
                ik[k] = k < keff ? iq[k - k0] : 0;
                ws += Wt[k];
            }
        }
    }
    if (SAMPLE) sample_tile(A, P.valid, P.q, p, keff, smem);
    if (!P.valid) return;
    // the colour sum: the gathers of each group of four slots are issued
    // together (slots past keff gather row 0 with weight 0; kmax > 0 implies
    // a kernel set with rows)
    if (A.image && kmax > 0) {
        if ((A.C & 3) == 0) {
            // four channels per load and store
            const int C4 = A.C >> 2;
            const auto a4 = gp(reinterpret_cast<const float4*>(A.attrs));
            const auto o4 = gp(reinterpret_cast<float4*>(A.image)) + p * C4;
            for (int c = 0; c < C4; ++c) {
                float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int k0 = 0; k0 < KB; k0 += 4) {
                    if (k0 < kmax) {
                        float4 v[4];
#pragma unroll
                        for (int k = k0; k < k0 + 4 && k < KB; ++k) v[k - k0] = ld_f4(a4 + (size_t)ik[k] * C4 + c);
#pragma unroll
                        for (int k = k0; k < k0 + 4 && k < KB; ++k) {
                            acc.x = fmaf(Wt[k], v[k - k0].x, acc.x);
                            acc.y = fmaf(Wt[k], v[k - k0].y, acc.y);
                            acc.z = fmaf(Wt[k], v[k - k0].z, acc.z);
                            acc.w = fmaf(Wt[k], v[k - k0].w, acc.w);
                        }
                    }
                }
                st_f4(o4 + c, acc);
            }
        } else if (A.C == 3) {
            // rows of three channels: one three-dword load per kept kernel
            const auto at = gp(A.attrs);
            const auto img = gp(A.image);
            float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
            for (int k0 = 0; k0 < KB; k0 += 4) {
                if (k0 < kmax) {
                    float r[4][3];
#pragma unroll
                    for (int k = k0; k < k0 + 4; ++k) {
                        const auto row = at + (size_t)ik[k] * 3;
                        r[k - k0][0] = row[0];
                        r[k - k0][1] = row[1];
                        r[k - k0][2] = row[2];
                    }
#pragma unroll
                    for (int k = k0; k < k0 + 4; ++k) {
                        a0 = fmaf(Wt[k], r[k - k0][0], a0);
                        a1 = fmaf(Wt[k], r[k - k0][1], a1);
                        a2 = fmaf(Wt[k], r[k - k0][2], a2);
                    }
                }
            }
            img[p * 3] = a0;
            img[p * 3 + 1] = a1;
            img[p * 3 + 2] = a2;
        } else {
            const auto at = gp(A.attrs);
            const auto img = gp(A.image);
            for (int c = 0; c < A.C; ++c) {
                float acc = 0.f;
#pragma unroll
                for (int k0 = 0; k0 < KB; k0 += 4) {
                    if (k0 < kmax) {
                        float v[4];
#pragma unroll
                        for (int k = k0; k < k0 + 4 && k < KB; ++k) v[k - k0] = at[(size_t)ik[k] * A.C + c];
#pragma unroll
                        for (int k = k0; k < k0 + 4 && k < KB; ++k) acc = fmaf(Wt[k], v[k - k0], acc);
                    }
                }
                img[p * A.C + c] = acc;
            }
        }
    } else if (A.image) {
        for (int c = 0; c < A.C; ++c) gp(A.image)[p * A.C + c] = 0.f;
    }
    if (A.wsum) gp(A.wsum)[p] = ws;
    if (A.kept) write_kept(A, P.q, p, keff);
}

// --------------------------------------------------------------- backward
//
// Given G = dL/dC of the pixel, with the kept set fixed:
//   dL/dc_k = W_k G;  g_k = G . c_k;  dL/dm_k (direct) = g_k T_k;  dL/dE_k = -g_k W_k
//   with x = (l_k - l_m) s_m and Phi'(x) = exp(-x^2)/sqrt(pi):
//     dE_k/dm_m = Phi(x);  dE_k/dl_k = m_m Phi' s_m = -dE_k/dl_m;
//     dE_k/da_m = m_m Phi' (l_k - l_m) / (2 s_m)
//   dq = dL/dm * m; to camera space with V = M - l D' (App. A.1):
//     dq/dM = -S V,  dq/dS = -V V^T / 2,  dq/dD' = l S V
//     dl/dM = S D'/a, dl/dS = sym(D' V^T)/a, dl/dD' = (S V - l S D')/a
//     da/dS = D' D'^T, da/dD' = 2 S D'
//
// Reduction over pixels without float atomics in LDS: the pixel lanes leave
// per-pair scalars (dq, dl, da, W) in the list scratch, a counting sort in
// LDS orders the tile's (pixel, slot) pairs by kernel (16-bit indices in
// LDS), and lanes walk runs of pairs, gather their scalars, run the chain in
// FP64 and accumulate in registers; each (tile, kernel) then makes one global
// atomic add per output value.

__device__ __forceinline__ int hash_slot(int* s_hkey, int hmask, int rank) {
    int h = (int)(((uint32_t)rank * 2654435761u) >> 7) & hmask;
    for (int probe = 0; probe <= hmask; ++probe) {
        const int cur = atomicCAS(&s_hkey[h], -1, rank);
        if (cur == -1 || cur == rank) return h;
        h = (h + 1) & hmask;
    }
    return -1;
}

__device__ __forceinline__ double wave_sum(double x) {
    for (int off = WAVE / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// The chain for one (pixel, kernel) pair: camera-space gradient of the
// centre (out[0..2]) and of the symmetric inverse covariance (out[3..8],
// xx xy xz yy yz zz), and dL/dD' added to gD.  The peak depth
// l = D'^T S M / D'^T S D' is recomputed here in FP64 from the kernel's
// camera-space record.
__device__ __forceinline__ void pair_chain(const GeoRec& G, double D0, double D1, double D2, double dq,
                                           double dlt, double dat, double out[9], double gD[3]) {
    const double s0 = G.S[0], s1 = G.S[1], s2 = G.S[2], s3 = G.S[3], s4 = G.S[4], s5 = G.S[5];
    const double SD0 = s0 * D0 + s1 * D1 + s2 * D2;
    const double SD1 = s1 * D0 + s3 * D1 + s4 * D2;
    const double SD2 = s2 * D0 + s4 * D1 + s5 * D2;
    const double ia = rcp_pos(D0 * SD0 + D1 * SD1 + D2 * SD2);
    const double l = (G.M[0] * SD0 + G.M[1] * SD1 + G.M[2] * SD2) * ia;
    const double V0 = G.M[0] - l * D0, V1 = G.M[1] - l * D1, V2 = G.M[2] - l * D2;
    const double SV0 = s0 * V0 + s1 * V1 + s2 * V2;
    const double SV1 = s1 * V0 + s3 * V1 + s4 * V2;
    const double SV2 = s2 * V0 + s4 * V1 + s5 * V2;
    const double dlk = dlt * ia;
    const double hq = -0.5 * dq;
    out[0] = -dq * SV0 + dlk * SD0;
    out[1] = -dq * SV1 + dlk * SD1;
    out[2] = -dq * SV2 + dlk * SD2;
    out[3] = hq * V0 * V0 + dlk * D0 * V0 + dat * D0 * D0;
    out[4] = hq * V0 * V1 + dlk * 0.5 * (D0 * V1 + D1 * V0) + dat * D0 * D1;
    out[5] = hq * V0 * V2 + dlk * 0.5 * (D0 * V2 + D2 * V0) + dat * D0 * D2;
    out[6] = hq * V1 * V1 + dlk * D1 * V1 + dat * D1 * D1;
    out[7] = hq * V1 * V2 + dlk * 0.5 * (D1 * V2 + D2 * V1) + dat * D1 * D2;
    out[8] = hq * V2 * V2 + dlk * D2 * V2 + dat * D2 * D2;
    gD[0] += dq * l * SV0 + dlk * (SV0 - l * SD0) + 2.0 * dat * SD0;
    gD[1] += dq * l * SV1 + dlk * (SV1 - l * SD1) + 2.0 * dat * SD1;
    gD[2] += dq * l * SV2 + dlk * (SV2 - l * SD2) + 2.0 * dat * SD2;
}

// The same chain summed over a run of pairs of one kernel.  The centre's
// gradient and dL/dD' are linear in S: per pair they are S (-dq V + dlk D)
// and S (dq l V + dlk (V - l D) + 2 dat D), so the run sums the vectors
// in uM and uD and applies S once (run_close).  The inverse covariance's
// gradient hq V V^T + dlk sym(D V^T) + dat D D^T is P_i V_j + Q_i D_j with
// P = hq V + dlk D / 2 and Q = dlk V / 2 + dat D, added to outS (xx xy xz
// yy yz zz).
__device__ __forceinline__ void pair_chain_run(const GeoRec& G, double D0, double D1, double D2, double dq,
                                               double dlt, double dat, double uM[3], double uD[3], float outS[6]) {
    const double s0 = G.S[0], s1 = G.S[1], s2 = G.S[2], s3 = G.S[3], s4 = G.S[4], s5 = G.S[5];
    const double SD0 = s0 * D0 + s1 * D1 + s2 * D2;
    const double SD1 = s1 * D0 + s3 * D1 + s4 * D2;
    const double SD2 = s2 * D0 + s4 * D1 + s5 * D2;
    const double ia = rcp_pos(D0 * SD0 + D1 * SD1 + D2 * SD2);
    const double l = (G.M[0] * SD0 + G.M[1] * SD1 + G.M[2] * SD2) * ia;
    const double V0 = G.M[0] - l * D0, V1 = G.M[1] - l * D1, V2 = G.M[2] - l * D2;
    const double dlk = dlt * ia;
    uM[0] += dlk * D0 - dq * V0;
    uM[1] += dlk * D1 - dq * V1;
    uM[2] += dlk * D2 - dq * V2;
    const double c1 = dq * l + dlk, c2 = 2.0 * dat - dlk * l;
    uD[0] += c1 * V0 + c2 * D0;
    uD[1] += c1 * V1 + c2 * D1;
    uD[2] += c1 * V2 + c2 * D2;
    const double hq = -0.5 * dq, hl = 0.5 * dlk;
    const double P0 = hq * V0 + hl * D0, P1 = hq * V1 + hl * D1, P2 = hq * V2 + hl * D2;
    const double Q0 = hl * V0 + dat * D0, Q1 = hl * V1 + dat * D1, Q2 = hl * V2 + dat * D2;
    outS[0] += (float)(P0 * V0 + Q0 * D0);
    outS[1] += (float)(P0 * V1 + Q0 * D1);
    outS[2] += (float)(P0 * V2 + Q0 * D2);
    outS[3] += (float)(P1 * V1 + Q1 * D1);
    outS[4] += (float)(P1 * V2 + Q1 * D2);
    outS[5] += (float)(P2 * V2 + Q2 * D2);
}

// The end of a run: the centre's gradient S uM into out[0..2], and S uD
// added to gD.
__device__ __forceinline__ void run_close(const GeoRec& G, const double uM[3], const double uD[3], float out[3],
                                          double gD[3]) {
    const double s0 = G.S[0], s1 = G.S[1], s2 = G.S[2], s3 = G.S[3], s4 = G.S[4], s5 = G.S[5];
    out[0] = (float)(s0 * uM[0] + s1 * uM[1] + s2 * uM[2]);
    out[1] = (float)(s1 * uM[0] + s3 * uM[1] + s4 * uM[2]);
    out[2] = (float)(s2 * uM[0] + s4 * uM[1] + s5 * uM[2]);
    gD[0] += s0 * uD[0] + s1 * uD[1] + s2 * uD[2];
    gD[1] += s1 * uD[0] + s3 * uD[1] + s4 * uD[2];
    gD[2] += s2 * uD[0] + s4 * uD[1] + s5 * uD[2];
}

// Pairs of a lane's chunk whose loads the tile reduction issues together.
constexpr int RED_BATCH = 4;

// Attribute channels per reduction pass: fewer at the deepest K-buffer, so
// that the partial sums and the pair indices fit 64 KB of LDS.
__host__ __device__ constexpr int red_ch(int KB) { return KB >= 64 ? 4 : 8; }

// Whether the reduction stages the tile's upstream gradient in LDS (4
// channels per pixel slot): with at most 4 channels and all but the deepest
// K-buffer, where the 4 KB keep three workgroups per CU.  Wider gradients
// are read from global memory pair by pair.
constexpr int GRAD_STAGE_CH = 4;
__host__ __device__ constexpr bool red_stage_grad(int KB, int max_c) { return KB < 64 && max_c <= GRAD_STAGE_CH; }

// LDS of the tile reduction: the hash table (keys, pair counts and offsets,
// hcap ints each), later reused for the
// reduction's partial sums (head and tail runs of every lane, nv values
// each: the 9 geometric ones and one pass's channels); then the tile's pairs
// in kernel order as 16-bit indices (256 * KB of them); then, when staged,
// the tile's upstream gradient (GRAD_STAGE_CH floats per pixel slot).
__host__ __device__ constexpr int bwd_partial_values(int KB, bool narrow) {
    return 9 + (narrow ? GRAD_STAGE_CH : red_ch(KB));
}

__host__ __device__ inline size_t bwd_table_bytes(int hcap, int nv) {
    const size_t table = (size_t)hcap * 3 * sizeof(int);
    const size_t partials = (size_t)TILE_THREADS * (2 * nv * sizeof(float) + 4 * sizeof(int));
    return ((table > partials ? table : partials) + 15) & ~(size_t)15;
}

size_t bwd_lds_bytes(int hcap, int KB, int max_c) {
    const size_t grad = red_stage_grad(KB, max_c) ? (size_t)TILE_THREADS * GRAD_STAGE_CH * sizeof(float) : 0;
    const size_t red =
        bwd_table_bytes(hcap, bwd_partial_values(KB, max_c <= GRAD_STAGE_CH)) + (size_t)TILE_THREADS * KB * sizeof(uint16_t) +
        grad;
    const size_t pix = (size_t)TILE_THREADS * KB * sizeof(float);   // the pixel phase's g_k T_k
    return red > pix ? red : pix;
}

// The original index of the kernel of a rank (the accumulators are kept in
// original order, so the epilogue reads and writes every array in order).
__device__ __forceinline__ size_t kernel_index(const TraceArgs& A, int rank) {
    return (gp(A.geo) + rank)->idx;
}

// Add one kernel's partial sums to global memory: the 9 geometric values
// (pass 0 only) and attribute channels c0 .. c0+nc-1, at the kernel's
// original index n.
template <int NCH>
__device__ __forceinline__ void flush_values(const TraceArgs& A, size_t n, const float* v, bool geom, int c0,
                                             int nc) {
    // v: the 9 geometric values, then nc <= NCH channels
    if (geom) {
#pragma unroll
        for (int q = 0; q < 3; ++q) global_add(&A.gM[n * 3 + q], v[q]);
#pragma unroll
        for (int q = 0; q < 6; ++q) global_add(&A.gS[n * 6 + q], v[3 + q]);
    }
#pragma unroll
    for (int q = 0; q < NCH; ++q)
        if (q < nc) global_add(&A.gA[n * A.C + c0 + q], v[9 + q]);
}

// Backward, pixel phase, pair loop of one lane's pixel (list index q, kept
// count keff, the wave's largest kept count kmax; l_k in lk, dE_k in dE, its
// g_k T_k at s_dmd[k * 256 + lane]).  m streams from the list (slot m+1 is
// loaded while slot m is computed); after the sums over k, slot m's scalars
// are complete except the k-side part of dL/dl, which goes to its own list at
// the end:
//   dq = (g_m T_m + sum_k dE_k Phi_km) m_m,  dl = -s_m sum_k dx_km (+ dl[m] later),
//   da = sum_k dx_km d_km / (2 s_m),  W = T_m m_m,
// with dx_km = dE_k m_m Phi'(x_km), x_km = d_km s_m, d_km = l_k - l_m.
template <int KB>
__device__ __forceinline__ void bwd_pair_loop(const TraceArgs& A, size_t q, int keff, int kmax, const float* s_dmd,
                                              const double (&lk)[KB], const float (&dE)[KB]) {
    const size_t S = A.S;
    const int tid = threadIdx.x;
    const auto pl = gp(A.kl_l) + q;
    const auto pm = gp(A.kl_m) + q;
    const auto ps = gp(A.kl_s) + q;
    const auto pT = gp(A.kl_T) + q;
    const auto pbw = gp(A.bw) + q;
    float dl[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) dl[k] = 0.f;
    double ln = keff > 0 ? pl[0] : 0.0;
    float mn = keff > 0 ? pm[0] : 0.f, sn = keff > 0 ? ps[0] : 1.f, tn = keff > 0 ? pT[0] : 0.f;
    for (int m = 0; m < kmax; ++m) {
        const bool in = m < keff;
        const size_t o = (size_t)m * S;
        const double lm = ln;
        const float mm = mn, sm = sn, tm = tn;
        const bool nin = m + 1 < keff;
        ln = nin ? pl[o + S] : 0.0;
        mn = nin ? pm[o + S] : 0.f;
        sn = nin ? ps[o + S] : 1.f;
        tn = nin ? pT[o + S] : 0.f;
        // dx_km = dE_k e_km m_m / sqrt(pi): the factor m_m / sqrt(pi) of slot
        // m is applied once to the sums over k
        const float sms = sm * SQRT_LOG2E, mmc = mm * INV_SQRT_PI, mcs = mmc * sm;
        float acc_dm = 0.f, acc_t = 0.f, acc_td = 0.f;
#pragma unroll
        for (int k0 = 0; k0 < KB; k0 += 4) {
            if (k0 < kmax) {
#pragma unroll
                for (int k = k0; k < k0 + 4 && k < KB; ++k) {
                    const float d = (float)(lk[k] - lm);
                    const float xs = d * sms;
                    const float ex = gauss_scaled(xs);
                    acc_dm = fmaf(dE[k], phi_from(xs, ex), acc_dm);
                    const float t = dE[k] * ex;
                    dl[k] = fmaf(t, mcs, dl[k]);
                    acc_t += t;
                    acc_td = fmaf(t, d, acc_td);
                }
            }
        }
        if (in) {
            const float dmd_m = s_dmd[m * TILE_THREADS + tid];
            st_f4(pbw + o, make_float4((dmd_m + acc_dm) * mm, -sm * (mmc * acc_t), (mmc * acc_td) * (0.5f / sm),
                                       tm * mm));
        }
    }
    // the k-side part of dL/dl of each slot
    const auto pbl = gp(A.bwl) + q;
#pragma unroll
    for (int k = 0; k < KB; ++k)
        if (k < keff) pbl[(size_t)k * S] = dl[k];
}

// Backward, pixel phase: per-pair scalars (dq, dl, da, W) into the scratch list.
template <int KB>
__device__ __forceinline__ void bwd_pix_body(const TraceArgs& A, int tile, float* s_dmd) {
    const int ntx = (A.W + TILE - 1) / TILE;
    const PixelCtx P = pixel_at(tile, balanced_slot(A, tile, ntx), ntx, A.H, A.W, A.cx, A.cy);
    const size_t S = A.S;
    const int C = A.C;

    const int keff = P.valid ? gp(A.keff)[P.q] : 0;
    const int kmax = wave_max_keff(keff);
    const size_t p = (size_t)P.pi * A.W + P.pj;
    const auto pl = gp(A.kl_l) + P.q;
    const auto pm = gp(A.kl_m) + P.q;
    const auto pT = gp(A.kl_T) + P.q;
    const auto pi = gp(A.kl_i) + P.q;
    const auto Gp = gp(A.grad_image) + p * C;

    double lk[KB];
    float dE[KB];
    int ik[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        lk[k] = 0.0;
        dE[k] = 0.f;
        ik[k] = 0;
        if (k < keff) {
            lk[k] = pl[(size_t)k * S];
            ik[k] = pi[(size_t)k * S];
        }
    }
    // g_k = G . c_k; the gathers of each group of four slots are issued
    // together (slots past keff gather row 0, unused; kmax > 0 implies a
    // kernel set with rows)
    float g[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) g[k] = 0.f;
    if (kmax > 0) {
        if ((C & 3) == 0) {
            const auto G4 = gp(reinterpret_cast<const float4*>(A.grad_image)) + p * (C >> 2);
            const auto A4 = gp(reinterpret_cast<const float4*>(A.attrs));
            const int C4 = C >> 2;
            for (int c = 0; c < C4; ++c) {
                float4 Gc = make_float4(0.f, 0.f, 0.f, 0.f);
                if (keff > 0) Gc = ld_f4(G4 + c);
#pragma unroll
                for (int k0 = 0; k0 < KB; k0 += 4) {
                    if (k0 < kmax) {
                        float4 a[4];
#pragma unroll
                        for (int k = k0; k < k0 + 4 && k < KB; ++k) a[k - k0] = ld_f4(A4 + (size_t)ik[k] * C4 + c);
#pragma unroll
                        for (int k = k0; k < k0 + 4 && k < KB; ++k)
                            g[k] = fmaf(Gc.x, a[k - k0].x,
                                        fmaf(Gc.y, a[k - k0].y, fmaf(Gc.z, a[k - k0].z, fmaf(Gc.w, a[k - k0].w, g[k]))));
                    }
                }
            }
        } else if (C == 3) {
            // rows of three channels: one three-dword load per kept kernel
            const auto at = gp(A.attrs);
            const float G0 = keff > 0 ? Gp[0] : 0.f, G1 = keff > 0 ? Gp[1] : 0.f, G2 = keff > 0 ? Gp[2] : 0.f;
#pragma unroll
            for (int k0 = 0; k0 < KB; k0 += 4) {
                if (k0 < kmax) {
                    float r[4][3];
#pragma unroll
                    for (int k = k0; k < k0 + 4; ++k) {
                        const auto row = at + (size_t)ik[k] * 3;
                        r[k - k0][0] = row[0];
                        r[k - k0][1] = row[1];
                        r[k - k0][2] = row[2];
                    }
#pragma unroll
                    for (int k = k0; k < k0 + 4; ++k)
                        g[k] = fmaf(G0, r[k - k0][0], fmaf(G1, r[k - k0][1], fmaf(G2, r[k - k0][2], g[k])));
                }
            }
        } else {
            const auto at = gp(A.attrs);
            for (int c = 0; c < C; ++c) {
                const float Gc = keff > 0 ? Gp[c] : 0.f;
#pragma unroll
                for (int k0 = 0; k0 < KB; k0 += 4) {
                    if (k0 < kmax) {
                        float a[4];
#pragma unroll
                        for (int k = k0; k < k0 + 4 && k < KB; ++k) a[k - k0] = at[(size_t)ik[k] * C + c];
#pragma unroll
                        for (int k = k0; k < k0 + 4 && k < KB; ++k) g[k] = fmaf(Gc, a[k - k0], g[k]);
                    }
                }
            }
        }
    }
    // the ablations stop the path through T (dE) or the direct factor e^q (dmd)
    const bool keep_T = !(A.grad_mode & 1), keep_rho = !(A.grad_mode & 2);
    // g_k T_k waits in LDS (slot k of the lane at s_dmd[k * 256 + lane]) for
    // the pass over m = k
    const int tid = threadIdx.x;
#pragma unroll
    for (int k0 = 0; k0 < KB; k0 += 4) {
        if (k0 < kmax) {
            // T_k and e^{q_k} of four slots, loaded together
            float Tq[4], Mq[4];
#pragma unroll
            for (int k = k0; k < k0 + 4; ++k) {
                const size_t o = (size_t)(k < kmax ? k : kmax - 1) * S;
                Tq[k - k0] = pT[o];
                Mq[k - k0] = pm[o];
            }
#pragma unroll
            for (int k = k0; k < k0 + 4; ++k) {
                const float T = Tq[k - k0];
                dE[k] = keep_T && k < keff ? -g[k] * (T * Mq[k - k0]) : 0.f;
                if (k < keff) s_dmd[k * TILE_THREADS + tid] = keep_rho ? g[k] * T : 0.f;
            }
        }
    }
    bwd_pair_loop<KB>(A, P.q, keff, kmax, s_dmd, lk, dE);
}

// Forward and the backward's pixel phase of a tile in one pass over its
// pixels, for a call that asks for both with the upstream gradient given:
// the blend (transmittance sums, weights, colour sum), then, with the kept
// depths, transmittances and weights still in registers and the attribute
// rows of the colour sum also giving g_k = G . c_k, the backward's dE_k and
// pair loop.  Its outputs are those of the blend and of the pixel phase.
template <int KB>
__device__ __forceinline__ void fwdbwd_pix_body(const TraceArgs& A, int tile, float* s_dmd) {
    const int ntx = (A.W + TILE - 1) / TILE;
    const PixelCtx P = pixel_at(tile, balanced_slot(A, tile, ntx), ntx, A.H, A.W, A.cx, A.cy);
    const size_t S = A.S;
    const int C = A.C;
    const int keff = P.valid ? gp(A.keff)[P.q] : 0;
    const int kmax = wave_max_keff(keff);
    const size_t p = (size_t)P.pi * A.W + P.pj;
    const auto pm = gp(A.kl_m) + P.q;
    double lk[KB];
    float E[KB];
    blend_sums<KB>(A, P.q, keff, kmax, lk, E);   // the blend's sums, as in blend_body
    // T_k waits in LDS (where g_k T_k goes later), W_k = T_k e^{q_k} in dE
    // until dE_k = -g_k W_k replaces it, and the original indices
    const int tid = threadIdx.x;
    float dE[KB];
    int ik[KB];
    float ws = 0.f;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        dE[k] = 0.f;
        ik[k] = 0;
    }
#pragma unroll
    for (int k0 = 0; k0 < KB; k0 += 4) {
        if (k0 < kmax) {
            float mq[4];
            int iq[4];
#pragma unroll
            for (int k = k0; k < k0 + 4; ++k) {
                const size_t o = (size_t)(k < kmax ? k : kmax - 1) * S;
                mq[k - k0] = pm[o];
                iq[k - k0] = gp(A.kl_i)[o + P.q];
            }
#pragma unroll
            for (int k = k0; k < k0 + 4; ++k) {
                const float T = expf(-E[k]);
                if (k < keff) {
                    gp(A.kl_T)[(size_t)k * S + P.q] = T;
                    s_dmd[k * TILE_THREADS + tid] = T;
                }
                dE[k] = k < keff ? T * mq[k - k0] : 0.f;
                ik[k] = k < keff ? iq[k - k0] : 0;
                ws += dE[k];
            }
        }
    }
    // dE_k = -g_k W_k and g_k T_k (as in bwd_pix_body, with the ablations)
    const bool keep_T = !(A.grad_mode & 1), keep_rho = !(A.grad_mode & 2);
    auto finish = [&](int k, float gk) {
        dE[k] = keep_T && k < keff ? -gk * dE[k] : 0.f;
        if (k < keff) s_dmd[k * TILE_THREADS + tid] = keep_rho ? gk * s_dmd[k * TILE_THREADS + tid] : 0.f;
    };
    // the colour sum (weights W_k in dE; slots past keff gather row 0 with
    // weight 0), and g_k = G . c_k; the upstream gradient is read only at
    // pixels with kept kernels, which lie in the image
    const bool img = A.image != nullptr && P.valid;
    if (kmax > 0 && C == 3) {
        // three channels: the rows of the colour sum give g_k too
        const auto at = gp(A.attrs);
        const auto Gp = gp(A.grad_image) + p * 3;
        const float G0 = keff > 0 ? Gp[0] : 0.f, G1 = keff > 0 ? Gp[1] : 0.f, G2 = keff > 0 ? Gp[2] : 0.f;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
        for (int k0 = 0; k0 < KB; k0 += 4) {
            if (k0 < kmax) {
                float r[4][3];
#pragma unroll
                for (int k = k0; k < k0 + 4; ++k) {
                    const auto row = at + (size_t)ik[k] * 3;
                    r[k - k0][0] = row[0];
                    r[k - k0][1] = row[1];
                    r[k - k0][2] = row[2];
                }
#pragma unroll
                for (int k = k0; k < k0 + 4; ++k) {
                    a0 = fmaf(dE[k], r[k - k0][0], a0);
                    a1 = fmaf(dE[k], r[k - k0][1], a1);
                    a2 = fmaf(dE[k], r[k - k0][2], a2);
                    finish(k, fmaf(G0, r[k - k0][0], fmaf(G1, r[k - k0][1], G2 * r[k - k0][2])));
                }
            }
        }
        if (img) {
            const auto out = gp(A.image) + p * 3;
            out[0] = a0;
            out[1] = a1;
            out[2] = a2;
        }
    } else if (kmax > 0) {
        // other channel counts: the colour sum channel by channel, then g_k
        // four slots at a time over all channels (a second gather of the
        // rows; one channel per load keeps the registers of the pair loop's
        // kernel free of spills)
        const auto at = gp(A.attrs);
        const auto Gp = gp(A.grad_image) + p * C;
        for (int c = 0; c < C; ++c) {
            float acc = 0.f;
#pragma unroll
            for (int k0 = 0; k0 < KB; k0 += 4) {
                if (k0 < kmax) {
                    float v[4];
#pragma unroll
                    for (int k = k0; k < k0 + 4; ++k) v[k - k0] = at[(size_t)ik[k] * C + c];
#pragma unroll
                    for (int k = k0; k < k0 + 4; ++k) acc = fmaf(dE[k], v[k - k0], acc);
                }
            }
            if (img) gp(A.image)[p * C + c] = acc;
        }
#pragma unroll
        for (int k0 = 0; k0 < KB; k0 += 4) {
            if (k0 < kmax) {
                float g4[4] = {0.f, 0.f, 0.f, 0.f};
                for (int c = 0; c < C; ++c) {
                    const float Gc = keff > 0 ? Gp[c] : 0.f;
#pragma unroll
                    for (int k = k0; k < k0 + 4; ++k) g4[k - k0] = fmaf(Gc, at[(size_t)ik[k] * C + c], g4[k - k0]);
                }
#pragma unroll
                for (int k = k0; k < k0 + 4; ++k) finish(k, g4[k - k0]);
            }
        }
    } else if (img) {
        for (int c = 0; c < C; ++c) gp(A.image)[p * C + c] = 0.f;
    }
    if (A.wsum && P.valid) gp(A.wsum)[p] = ws;
    if (A.kept && P.valid) write_kept(A, P.q, p, keff);
    bwd_pair_loop<KB>(A, P.q, keff, kmax, s_dmd, lk, dE);
}

// Backward, tile phase: group the tile's pairs by kernel and reduce them.
// NARROW: every item of the launch has at most GRAD_STAGE_CH channels (one
// pass of that many channels; the upstream gradient staged in LDS below the
// deepest K-buffer).
// The lane's pixel is pixel_of(tile); rk[k]: the rank of its slot k, -1 past
// its kept count.
template <int KB, bool NARROW>
__device__ __forceinline__ void bwd_red_body(const TraceArgs& A, int hcap, int tile, unsigned char* smem,
                                             const int (&rk)[KB]) {
    constexpr bool stage = NARROW && red_stage_grad(KB, GRAD_STAGE_CH);
    __shared__ double s_red[TILE_THREADS / WAVE][3];
    __shared__ int s_wtot[TILE_THREADS / WAVE];
    const int tid = threadIdx.x;
    const int ntx = (A.W + TILE - 1) / TILE;
    const PixelCtx P = pixel_of(tile, ntx, A.H, A.W, A.cx, A.cy);
    const size_t S = A.S;
    const int C = A.C;
    int* s_hkey = reinterpret_cast<int*>(smem);
    int* s_cnt = s_hkey + hcap;
    int* s_off = s_cnt + hcap;
    for (int i = tid; i < hcap; i += TILE_THREADS) {
        s_hkey[i] = -1;
        s_cnt[i] = 0;
    }
    const int keff = P.valid ? gp(A.keff)[P.q] : 0;
    const size_t p = (size_t)P.pi * A.W + P.pj;
    const float* Gp = A.grad_image + p * C;
    const size_t q0 = (size_t)tile * TILE_THREADS;            // the tile's first list index
    constexpr int RED_CH = NARROW ? GRAD_STAGE_CH : red_ch(KB);   // attribute channels per reduction pass
    constexpr int RED_NV = 9 + RED_CH;           // values per partial sum (registers)
    constexpr int nvs = bwd_partial_values(KB, NARROW);   // values per partial sum in LDS (= RED_NV)
    uint16_t* s_pair = reinterpret_cast<uint16_t*>(smem + bwd_table_bytes(hcap, nvs));
    // the tile's upstream gradient (stage: C <= GRAD_STAGE_CH, one pass),
    // GRAD_STAGE_CH values per pixel slot
    float* s_g = reinterpret_cast<float*>(s_pair + (size_t)TILE_THREADS * KB);
    __syncthreads();   // table initialised

    // counting sort of the tile's pairs by kernel; sp[k] = table slot << 16 | position.
    // All first probes are issued back to back; collisions (rare at this load
    // factor) then probe on.
    int sp[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        sp[k] = -1;
        if (rk[k] >= 0) {
            const int h = (int)(((uint32_t)rk[k] * 2654435761u) >> 7) & (hcap - 1);
            const int cur = atomicCAS(&s_hkey[h], -1, rk[k]);
            sp[k] = (cur == -1 || cur == rk[k]) ? h : -2;
        }
    }
#pragma unroll
    for (int k = 0; k < KB; ++k)
        if (sp[k] == -2) sp[k] = hash_slot(s_hkey, hcap - 1, rk[k]);
#pragma unroll
    for (int k = 0; k < KB; ++k)
        if (sp[k] >= 0) sp[k] = (sp[k] << 16) | atomicAdd(&s_cnt[sp[k]], 1);
    __syncthreads();
    // exclusive scan s_cnt -> s_off: each lane sums its run of entries, the
    // wave scans the sums with shuffles, and one barrier exchanges the wave
    // totals
    {
        const int per = (hcap + TILE_THREADS - 1) / TILE_THREADS;
        const int lane = tid % WAVE, wave = tid / WAVE;
        int run = 0;
        for (int j = 0; j < per; ++j) {
            const int i = tid * per + j;
            if (i < hcap) run += s_cnt[i];
        }
        int inc = run;
        for (int off = 1; off < WAVE; off <<= 1) {
            const int y = __shfl_up(inc, off);
            if (lane >= off) inc += y;
        }
        if (lane == WAVE - 1) s_wtot[wave] = inc;
        __syncthreads();
        for (int w = 0; w < wave; ++w) inc += s_wtot[w];
        int base = inc - run;
        for (int j = 0; j < per; ++j) {
            const int i = tid * per + j;
            if (i < hcap) {
                s_off[i] = base;
                base += s_cnt[i];
            }
        }
    }
    __syncthreads();
    double gD[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        if (k < keff) {
            if (sp[k] >= 0) {
                // the pair (slot k, pixel tid) at its place in kernel order; bit
                // 15 marks the first pair of a kernel's run
                const int pos = sp[k] & 0xFFFF;
                s_pair[s_off[sp[k] >> 16] + pos] = (uint16_t)((pos == 0 ? 0x8000 : 0) | (k << 8) | tid);
            } else {
                // table full: this pair goes straight to global memory
                const size_t o = (size_t)k * S + P.q;
                const int rank = rk[k];
                const float4 sc = ld_f4(gp(A.bw) + o);
                const GeoRec G = load_geo(gp(A.geo) + rank);
                double out[9];
                pair_chain(G, P.u, P.v, (double)A.F, sc.x, sc.y + gp(A.bwl)[o], sc.z, out, gD);
                const size_t n = G.idx;
#pragma unroll
                for (int e = 0; e < 3; ++e) global_add(&A.gM[n * 3 + e], (float)out[e]);
#pragma unroll
                for (int e = 0; e < 6; ++e) global_add(&A.gS[n * 6 + e], (float)out[3 + e]);
                for (int c = 0; c < C; ++c) global_add(&A.gA[n * C + c], sc.w * gp(Gp)[c]);
            }
        }
    }
    __syncthreads();

    // Balanced segmented reduction.  Lane t takes an equal, contiguous chunk
    // of the tile's kernel-sorted pairs and sums runs of equal kernels.  A run
    // that lies inside the chunk is complete and is added to global memory at
    // once; the first and last runs of a chunk may continue in the neighbouring
    // chunks, so they go to LDS, and the lane where a kernel's run starts adds
    // up the continuation and flushes it: one global add per (tile, kernel,
    // value).  Pass 0 reduces the 9 geometric values and the first RED_CH
    // attribute channels, later passes the next RED_CH channels.
    const int ti0 = (tile / ntx) * TILE, tj0 = (tile % ntx) * TILE;
    const int n_pairs = s_off[hcap - 1] + s_cnt[hcap - 1];
    __syncthreads();   // the table's LDS becomes the partial-sum buffers
    float* s_head = reinterpret_cast<float*>(smem);
    float* s_tail = s_head + TILE_THREADS * nvs;
    int* s_hk = reinterpret_cast<int*>(s_tail + TILE_THREADS * nvs);
    int* s_tk = s_hk + TILE_THREADS;
    int* s_hn = s_tk + TILE_THREADS;            // the original indices of those kernels
    int* s_tn = s_hn + TILE_THREADS;
    const int per = (n_pairs + TILE_THREADS - 1) / TILE_THREADS;
    const int j0 = min(n_pairs, tid * per), j1 = min(n_pairs, j0 + per);
    // pair j in kernel order: its scalars gathered from the slot-major lists
    // (the chain's three only in pass 0); its kernel's rank where a run
    // starts, or at the chunk's first pair (-1: same kernel as before)
    struct Pair {
        float dq = 0.f, dl = 0.f, da = 0.f, w = 0.f;
        int rank = -1, pt = 0;
    };
    auto load_pair = [&](int j, bool geom) {
        const int e = s_pair[j];
        const size_t o = (size_t)((e >> 8) & 63) * S + q0 + (e & 255);
        Pair r;
        if (geom) {
            const float4 sc = ld_f4(gp(A.bw) + o);
            r.dq = sc.x;
            r.dl = sc.y + gp(A.bwl)[o];
            r.da = sc.z;
            r.w = sc.w;
        } else {
            r.dq = r.dl = r.da = 0.f;
            r.w = gp(reinterpret_cast<const float*>(A.bw + o))[3];
        }
        r.rank = ((e & 0x8000) || j == j0) ? gp(A.kl_r)[o] : -1;
        r.pt = e & 255;
        return r;
    };
    for (int c0 = 0; c0 == 0 || c0 < C; c0 += RED_CH) {
        const bool geom = c0 == 0;
        const int nc = max(0, min(RED_CH, C - c0));
        float acc[RED_NV];
#pragma unroll
        for (int q = 0; q < RED_NV; ++q) acc[q] = 0.f;
        int cur = -1, nseg = 0;
        size_t cur_n = 0;
        GeoRec G;
        double uM[3] = {0.0, 0.0, 0.0}, uD[3] = {0.0, 0.0, 0.0};   // the run's S-factored sums
        s_hk[tid] = -1;
        s_tk[tid] = -1;
        if (stage) {
            // the channels of the lane's own pixel (zeros past channel C and
            // outside the image): the pairs below read them from LDS
            float g[GRAD_STAGE_CH];
#pragma unroll
            for (int q = 0; q < GRAD_STAGE_CH; ++q) g[q] = (P.valid && q < nc) ? gp(Gp)[q] : 0.f;
            reinterpret_cast<float4*>(s_g)[tid] = make_float4(g[0], g[1], g[2], g[3]);
            __syncthreads();
        }
        // the run `cur` ends: the chunk's first run (it may continue from the
        // previous chunk) and its last (it may continue into the next) go to
        // LDS, a run inside the chunk is complete and is flushed
        auto close_run = [&](bool end) {
            if (geom) run_close(G, uM, uD, acc, gD);
            if (nseg == 0) {
                s_hk[tid] = cur;
                s_hn[tid] = (int)cur_n;
#pragma unroll
                for (int q = 0; q < RED_NV; ++q)
                    s_head[tid * nvs + q] = acc[q];
            } else if (end) {
                s_tk[tid] = cur;
                s_tn[tid] = (int)cur_n;
#pragma unroll
                for (int q = 0; q < RED_NV; ++q)
                    s_tail[tid * nvs + q] = acc[q];
            } else {
                flush_values<RED_CH>(A, cur_n, acc, geom, c0, nc);
            }
            ++nseg;
        };
        // the chunk in batches of RED_BATCH pairs: a batch's loads are all in
        // flight before its first pair is reduced
        for (int jb = j0; jb < j1; jb += RED_BATCH) {
            Pair bp[RED_BATCH];
#pragma unroll
            for (int b = 0; b < RED_BATCH; ++b) bp[b] = jb + b < j1 ? load_pair(jb + b, geom) : Pair{};
#pragma unroll
            for (int b = 0; b < RED_BATCH; ++b) {
                if (jb + b < j1) {
                    const Pair& r = bp[b];
                    if (r.rank >= 0 && r.rank != cur) {
                        if (cur >= 0) close_run(false);
#pragma unroll
                        for (int q = 0; q < RED_NV; ++q) acc[q] = 0.f;
#pragma unroll
                        for (int q = 0; q < 3; ++q) uM[q] = uD[q] = 0.0;
                        cur = r.rank;
                        if (geom) {
                            G = load_geo(gp(A.geo) + cur);
                            cur_n = G.idx;
                        } else {
                            cur_n = kernel_index(A, cur);
                        }
                    }
                    const int w = r.pt / WAVE, ln = r.pt % WAVE;
                    const int row = ti0 + (w >> 1) * 8 + (ln >> 3), col = tj0 + (w & 1) * 8 + (ln & 7);
                    if (geom)
                        pair_chain_run(G, (double)row - (double)A.cy, (double)col - (double)A.cx, (double)A.F, r.dq,
                                       r.dl, r.da, uM, uD, acc + 3);
                    if (stage) {
                        const float4 g4 = reinterpret_cast<const float4*>(s_g)[r.pt];
                        acc[9] = fmaf(r.w, g4.x, acc[9]);
                        acc[10] = fmaf(r.w, g4.y, acc[10]);
                        acc[11] = fmaf(r.w, g4.z, acc[11]);
                        acc[12] = fmaf(r.w, g4.w, acc[12]);
                    } else {
                        const auto Gq = gp(A.grad_image) + ((size_t)row * A.W + col) * C + c0;
                        if (nc == RED_CH && (C & 3) == 0) {
#pragma unroll
                            for (int q = 0; q < RED_CH; q += 4) {
                                const float4 g4 = ld_f4((gptr<const float4>)(Gq + q));
                                acc[9 + q] = fmaf(r.w, g4.x, acc[9 + q]);
                                acc[10 + q] = fmaf(r.w, g4.y, acc[10 + q]);
                                acc[11 + q] = fmaf(r.w, g4.z, acc[11 + q]);
                                acc[12 + q] = fmaf(r.w, g4.w, acc[12 + q]);
                            }
                        } else {
                            for (int q = 0; q < nc; ++q) acc[9 + q] = fmaf(r.w, Gq[q], acc[9 + q]);
                        }
                    }
                }
            }
        }
        if (cur >= 0) close_run(true);
        __syncthreads();
        // the lane where a kernel's run starts adds the continuation and flushes
        for (int which = 0; which < 2; ++which) {
            const int k = which == 0 ? s_hk[tid] : s_tk[tid];
            if (k < 0) continue;
            if (which == 0 && tid > 0) {
                const int prev = s_tk[tid - 1] >= 0 ? s_tk[tid - 1] : s_hk[tid - 1];
                if (prev == k) continue;                               // started in an earlier chunk
            }
            const float* own = (which == 0 ? s_head : s_tail) + tid * nvs;
            float sum[RED_NV];
#pragma unroll
            for (int q = 0; q < RED_NV; ++q) sum[q] = own[q];
            for (int t2 = tid + 1; t2 < TILE_THREADS && s_hk[t2] == k; ++t2) {
                if (which == 0 && s_tk[tid] >= 0) break;              // own head run ended in this chunk
#pragma unroll
                for (int q = 0; q < RED_NV; ++q)
                    sum[q] += s_head[t2 * nvs + q];
                if (s_tk[t2] >= 0) break;                             // the run ends inside chunk t2
            }
            flush_values<RED_CH>(A, (size_t)(which == 0 ? s_hn[tid] : s_tn[tid]), sum, geom, c0, nc);
        }
        __syncthreads();
    }

    // per-tile sum of dL/dD' (for the intrinsics), fixed order
    const int wave = tid / WAVE, lane = tid % WAVE;
    const double gx = wave_sum(gD[0]), gy = wave_sum(gD[1]), gz = wave_sum(gD[2]);
    if (lane == 0) {
        s_red[wave][0] = gx;
        s_red[wave][1] = gy;
        s_red[wave][2] = gz;
    }
    __syncthreads();
    if (tid < 3) {
        double sum = 0.0;
        for (int w = 0; w < TILE_THREADS / WAVE; ++w) sum += s_red[w][tid];
        gp(A.tileD)[(size_t)tile * 3 + tid] = sum;
    }
}

// ------------------------------------------------------- exact-integral mode
//
// The outer integral of Eq. 1 by quadrature for each pixel's kept set, next
// to the closed form of Eq. 8, both in FP64 (a diagnostic of the
// approximation, App. A.2).  Along the ray kernel m has density
// e^{q_m} g_m(t), g_m(t) = sqrt(a_m/pi) exp(-a_m (t - l_m)^2), whose running
// integral is the erf sum of Eq. 7; the transmittance is exp(-E(t)) and
//   W_m = int T(t) e^{q_m} g_m(t) dt
// is taken by the trapezoid rule on n_samples points over
// [min_m l_m - 9/sqrt(a_m), max_m l_m + 9/sqrt(a_m)] (D' units; the rule is
// invariant under the scaling of t).  One wave per pixel: each kept kernel
// is re-traced in FP64 from its record, lane j takes samples j, j + 64, ...,
// and the per-kernel sums are reduced across the wave.
constexpr int QUAD_BLOCKS_PER_TILE = TILE_THREADS / (TILE_THREADS / WAVE);   // a block: one pixel per wave

template <int KB>
__global__ __launch_bounds__(TILE_THREADS) void k_quadrature(GroupDev g, QuadOut out) {
    __shared__ double s_l[TILE_THREADS / WAVE][KB], s_a[TILE_THREADS / WAVE][KB], s_m[TILE_THREADS / WAVE][KB];
    const TraceArgs A = g.items[g.single].t;
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int tile = blockIdx.x / QUAD_BLOCKS_PER_TILE;
    const int slot = (blockIdx.x % QUAD_BLOCKS_PER_TILE) * (TILE_THREADS / WAVE) + w;
    const int ntx = (A.W + TILE - 1) / TILE;
    const PixelCtx P = pixel_at(tile, slot, ntx, A.H, A.W, A.cx, A.cy);
    if (!P.valid) return;                       // whole wave: one pixel per wave
    const size_t S = A.S;
    const int keff = A.keff[P.q];
    const size_t p = (size_t)P.pi * A.W + P.pj;
    if (lane < keff) {
        const int rank = A.kl_r[(size_t)lane * S + P.q];
        double l, q2, a;
        trace_one(A.rec[rank], P.u, P.v, l, q2, a);
        s_l[w][lane] = l;
        s_a[w][lane] = a;
        s_m[w][lane] = exp(-0.5 * q2);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double t0 = 0.0, t1 = 0.0, msum = 0.0;
    for (int m = 0; m < keff; ++m) {
        const double r = 9.0 / sqrt(s_a[w][m]);
        t0 = m == 0 ? s_l[w][m] - r : fmin(t0, s_l[w][m] - r);
        t1 = m == 0 ? s_l[w][m] + r : fmax(t1, s_l[w][m] + r);
        msum += s_m[w][m];
    }
    double acc[KB];
#pragma unroll
    for (int m = 0; m < KB; ++m) acc[m] = 0.0;
    if (keff > 0) {
        const int n = out.n_samples;
        const double h = (t1 - t0) / (double)(n - 1);
        for (int s = lane; s < n; s += WAVE) {
            const double t = t0 + h * (double)s;
            const double wgt = (s == 0 || s == n - 1) ? 0.5 * h : h;
            double E = 0.0;
            for (int m = 0; m < keff; ++m) E += s_m[w][m] * 0.5 * (1.0 + erf((t - s_l[w][m]) * sqrt(s_a[w][m])));
            const double T = exp(-E);
#pragma unroll
            for (int m = 0; m < KB; ++m) {
                if (m < keff) {
                    const double d = t - s_l[w][m];
                    acc[m] += wgt * T * s_m[w][m] * sqrt(s_a[w][m] / M_PI) * exp(-s_a[w][m] * d * d);
                }
            }
        }
    }
    double sum_exact = 0.0;
#pragma unroll
    for (int m = 0; m < KB; ++m) {
        if (m < keff) {
            const double v = wave_sum(acc[m]);
            sum_exact += v;
            if (lane == 0) out.w_exact[p * A.K + m] = v;
        }
    }
    // the closed form of Eq. 7-8 in FP64, lane m for kernel m
    for (int m = lane; m < A.K; m += WAVE) {
        double wa = 0.0;
        if (m < keff) {
            double E = 0.0;
            for (int j = 0; j < keff; ++j)
                E += s_m[w][j] * 0.5 * (1.0 + erf((s_l[w][m] - s_l[w][j]) * sqrt(s_a[w][j])));
            wa = exp(-E) * s_m[w][m];
        } else {
            out.w_exact[p * A.K + m] = 0.0;
        }
        out.w_approx[p * A.K + m] = wa;
        if (out.kept) out.kept[p * A.K + m] = m < keff ? A.kl_i[(size_t)m * S + P.q] : -1;
    }
    if (lane == 0) {
        out.total[2 * p] = sum_exact;
        out.total[2 * p + 1] = 1.0 - exp(-msum);
    }
}

// ------------------------------------------------------------------ kernels
// A workgroup takes a tile of the group, finds the tile's item and renders
// the item-local tile with a copy of the item's view.  The copy is read
// before the kernel's first store, so the compiler keeps the fields in scalar
// registers instead of re-reading the table after each store.
__device__ __forceinline__ TraceArgs item_view(const GroupDev& g, int& tile) {
    const int gt = g.tile0 + tile_of_block(g.order);
    const int item = g.single >= 0 ? g.single : g.tile_item[gt];
    const ItemDev* it = g.items + item;
    tile = gt - it->tile_start;
    return it->t;
}

// Waves per SIMD the select kernel must fit (a register cap for the
// compiler): three at a K-buffer of 32 keys, which would otherwise drop to
// two; seven and eight at 20 and 16 keys for the record scan (six and seven
// for the bin scan, whose bin entries take registers too; a tighter cap
// spills).
template <int KB, bool BINS>
constexpr int select_waves() { return KB == 32 ? 3 : KB == 20 ? (BINS ? 6 : 7) : KB == 16 ? (BINS ? 7 : 8) : 1; }

// BINS: the launch holds binned items, whose tiles' bins are sorted into the
// dynamic LDS s_rank (BIN_MAX entries) and scanned in place of every record;
// a launch without binned items compiles the record scan alone.
template <int KB, bool BINS>
__global__ __launch_bounds__(TILE_THREADS, (select_waves<KB, BINS>())) void k_select(GroupDev g) {
    extern __shared__ __align__(16) uint32_t s_rank[];
    int tile;
    const TraceArgs A = item_view(g, tile);
    const int blk = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    if constexpr (BINS) {
        const int n_bin = load_bin(A, tile, s_rank);
        if (n_bin >= 0) {
            select_body<KB, true>(A, tile, blk, s_rank, n_bin);
            return;
        }
    }
    select_body<KB, false>(A, tile, blk, nullptr, A.N);
}

// Tiles from which select's record scan runs one wave per workgroup: with
// fewer, all of a launch's blocks fit the chip's wave slots at once, and
// four-wave workgroups spread them evenly over the SIMDs.
constexpr int SELECT_WAVE_MIN_TILES = 2048;

// The record scan with one wave per workgroup: a workgroup is one 8x8
// block, so the slot of a wave that ends takes any waiting block.  (With a
// tile's four waves in one workgroup, a new tile needed a free slot on all
// four SIMDs at once, and the blocks' unequal scans left slots idle.)  The
// launch has four units per tile, dealt to the XCDs in bands like tiles.
template <int KB>
__global__ __launch_bounds__(WAVE, (select_waves<KB, false>())) void k_select_wave(GroupDev g) {
    const int unit = tile_of_block(g.order);     // tile * 4 + block
    const int gt = g.tile0 + unit / 4;
    const int item = g.single >= 0 ? g.single : g.tile_item[gt];
    const ItemDev* it = g.items + item;
    const TraceArgs A = it->t;
    select_body<KB, false>(A, gt - it->tile_start, unit % 4, nullptr, A.N);
}

template <int KB>
__global__ __launch_bounds__(TILE_THREADS) void k_blend(GroupDev g) {
    int tile;
    const TraceArgs A = item_view(g, tile);
    blend_body<KB, false>(A, tile, nullptr);
}

template <int KB>
__global__ __launch_bounds__(TILE_THREADS) void k_blend_sample(GroupDev g) {
    extern __shared__ __align__(16) unsigned char smem[];
    int tile;
    const TraceArgs A = item_view(g, tile);
    blend_body<KB, true>(A, tile, smem);
}

// The backward of a tile: the pixel phase leaves its per-pair scalars in the
// slot-major scratch lists, and after a workgroup barrier (which makes the
// workgroup's global writes visible to all its lanes) the tile reduction
// reads them back while they are still in the XCD's L2.  Waves per SIMD the
// register allocation must fit: three up to a K-buffer of 20 (a cap of 168
// VGPRs), two at 32; at 64 a tighter cap would spill.
template <int KB>
constexpr int bwd_waves() { return KB <= 20 ? 3 : KB <= 32 ? 2 : 1; }

// After the pixel phase: the ranks of the reduction's pairs are loaded while
// the other waves finish the pixel phase; at the workgroup barrier a tile
// without kept pairs stops (its sum of dL/dD' is zero), any other goes on to
// the tile reduction.
template <int KB, bool NARROW>
__device__ __forceinline__ void bwd_after_pix(const TraceArgs& A, int tile, int hcap, unsigned char* smem) {
    const int ntx = (A.W + TILE - 1) / TILE;
    const PixelCtx P = pixel_of(tile, ntx, A.H, A.W, A.cx, A.cy);
    const int keff = P.valid ? gp(A.keff)[P.q] : 0;
    int rk[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) rk[k] = k < keff ? gp(A.kl_r)[P.q + (size_t)k * A.S] : -1;
    if (!__syncthreads_or(keff > 0)) {
        if (threadIdx.x < 3) gp(A.tileD)[(size_t)tile * 3 + threadIdx.x] = 0.0;
        return;
    }
    bwd_red_body<KB, NARROW>(A, hcap, tile, smem, rk);
}

template <int KB, bool NARROW>
__global__ __launch_bounds__(TILE_THREADS, bwd_waves<KB>()) void k_bwd(GroupDev g, int hcap) {
    extern __shared__ __align__(16) unsigned char smem[];
    int tile;
    const TraceArgs A = item_view(g, tile);
    {
        // a tile without kept pairs has nothing to reduce; its sum of dL/dD' is zero
        const int ntx = (A.W + TILE - 1) / TILE;
        const PixelCtx P = pixel_of(tile, ntx, A.H, A.W, A.cx, A.cy);
        const int ke = P.valid ? gp(A.keff)[P.q] : 0;
        if (!__syncthreads_or(ke > 0)) {
            if (threadIdx.x < 3) gp(A.tileD)[(size_t)tile * 3 + threadIdx.x] = 0.0;
            return;
        }
    }
    bwd_pix_body<KB>(A, tile, reinterpret_cast<float*>(smem));
    bwd_after_pix<KB, NARROW>(A, tile, hcap, smem);
}

// Forward and backward of a tile in one workgroup (a call that asks for
// both, with the upstream gradient given).
template <int KB, bool NARROW>
__global__ __launch_bounds__(TILE_THREADS, bwd_waves<KB>()) void k_fwdbwd(GroupDev g, int hcap) {
    extern __shared__ __align__(16) unsigned char smem[];
    int tile;
    const TraceArgs A = item_view(g, tile);
    fwdbwd_pix_body<KB>(A, tile, reinterpret_cast<float*>(smem));
    bwd_after_pix<KB, NARROW>(A, tile, hcap, smem);
}

// Diagnostics: the device Phi on an array.
__global__ void k_phi(const float* __restrict__ x, float* __restrict__ y, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = phi_cdf(x[i]);
}

// ---------------------------------------------------------------- launch
int pick_kbuf(int K) {
    if (K <= 8) return 8;
    if (K <= 16) return 16;
    if (K <= 20) return 20;
    if (K <= 32) return 32;
    return 64;
}

int table_capacity(int C) {
    (void)C;
    return 1024;   // distinct kernels one tile can reduce in LDS; more go to global atomics
}

template <int KB>
static hipError_t run_kb(int which, const GroupDev& g, hipStream_t s, int max_c = 1) {
    const int nt = g.n_tiles;
    if (nt <= 0) return hipSuccess;
    if (which == 0) {
        if (g.bins)
            hipLaunchKernelGGL((k_select<KB, true>), dim3(nt), dim3(TILE_THREADS), BIN_MAX * sizeof(uint32_t), s, g);
        else if (nt >= SELECT_WAVE_MIN_TILES)
            hipLaunchKernelGGL((k_select_wave<KB>), dim3(4 * nt), dim3(WAVE), 0, s, g);
        else
            hipLaunchKernelGGL((k_select<KB, false>), dim3(nt), dim3(TILE_THREADS), 0, s, g);
    } else if (which == 1) {
        hipLaunchKernelGGL(k_blend<KB>, dim3(nt), dim3(TILE_THREADS), 0, s, g);
    } else if (which == 2) {
        const int hcap = table_capacity(0);
        if (max_c <= GRAD_STAGE_CH)
            hipLaunchKernelGGL((k_bwd<KB, true>), dim3(nt), dim3(TILE_THREADS), bwd_lds_bytes(hcap, KB, max_c), s, g,
                               hcap);
        else
            hipLaunchKernelGGL((k_bwd<KB, false>), dim3(nt), dim3(TILE_THREADS), bwd_lds_bytes(hcap, KB, max_c), s, g,
                               hcap);
    } else if (which == 5) {
        const int hcap = table_capacity(0);
        if (max_c <= GRAD_STAGE_CH)
            hipLaunchKernelGGL((k_fwdbwd<KB, true>), dim3(nt), dim3(TILE_THREADS), bwd_lds_bytes(hcap, KB, max_c), s, g,
                               hcap);
        else
            hipLaunchKernelGGL((k_fwdbwd<KB, false>), dim3(nt), dim3(TILE_THREADS), bwd_lds_bytes(hcap, KB, max_c), s,
                               g, hcap);
    } else {
        hipLaunchKernelGGL(k_blend_sample<KB>, dim3(nt), dim3(TILE_THREADS), sample_lds_bytes(max_c), s, g);
    }
    return hipGetLastError();
}

static hipError_t dispatch(int which, const GroupDev& g, int kb, hipStream_t s, int max_c = 1) {
    switch (kb) {
        case 8: return run_kb<8>(which, g, s, max_c);
        case 16: return run_kb<16>(which, g, s, max_c);
        case 20: return run_kb<20>(which, g, s, max_c);
        case 32: return run_kb<32>(which, g, s, max_c);
        default: return run_kb<64>(which, g, s, max_c);
    }
}

hipError_t launch_select(const GroupDev& g, int kb, hipStream_t s) { return dispatch(0, g, kb, s); }
hipError_t launch_blend(const GroupDev& g, int kb, hipStream_t s) { return dispatch(1, g, kb, s); }
hipError_t launch_bwd(const GroupDev& g, int kb, int max_c, hipStream_t s) { return dispatch(2, g, kb, s, max_c); }
hipError_t launch_fwdbwd(const GroupDev& g, int kb, int max_c, hipStream_t s) { return dispatch(5, g, kb, s, max_c); }
hipError_t launch_blend_sample(const GroupDev& g, int kb, int max_c, hipStream_t s) {
    return dispatch(4, g, kb, s, max_c);
}

hipError_t launch_quadrature(const GroupDev& g, int kb, const QuadOut& out, hipStream_t s) {
    const int nb = g.n_tiles * QUAD_BLOCKS_PER_TILE;
    if (nb <= 0) return hipSuccess;
    switch (kb) {
        case 8: hipLaunchKernelGGL(k_quadrature<8>, dim3(nb), dim3(TILE_THREADS), 0, s, g, out); break;
        case 16: hipLaunchKernelGGL(k_quadrature<16>, dim3(nb), dim3(TILE_THREADS), 0, s, g, out); break;
        case 20: hipLaunchKernelGGL(k_quadrature<20>, dim3(nb), dim3(TILE_THREADS), 0, s, g, out); break;
        case 32: hipLaunchKernelGGL(k_quadrature<32>, dim3(nb), dim3(TILE_THREADS), 0, s, g, out); break;
        default: hipLaunchKernelGGL(k_quadrature<64>, dim3(nb), dim3(TILE_THREADS), 0, s, g, out); break;
    }
    return hipGetLastError();
}

hipError_t launch_phi(const float* x, float* y, int n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_phi, dim3((n + 255) / 256), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

}  // namespace voge
