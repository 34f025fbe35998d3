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
    for (int d = 0; d < 3; ++d) {
        M0[d] = (double)means[3 * (size_t)n + d];
        ok = ok && isfinite(M0[d]);
    }
    for (int e = 0; e < 6; ++e) {
        Sig[e] = (double)covs[6 * (size_t)n + e];
        ok = ok && isfinite(Sig[e]);
    }
    return ok;
}

__global__ void k_prep_keys(const float* __restrict__ means, const float* __restrict__ covs, int N, CamDev cam,
                            double rad2, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                            int* __restrict__ status) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double M0[3], Sig[6], S0[6];
    uint32_t key = KEY_CULLED;
    const bool finite = load_kernel(means, covs, n, M0, Sig);
    if (!finite) {
        atomicOr(status, ST_NONFINITE);
    } else if (!spd_inverse6(Sig, S0)) {
        atomicOr(status, ST_NOTSPD);
    } else {
        const double r0 = cam.R[6], r1 = cam.R[7], r2 = cam.R[8];
        const double Mz = r0 * M0[0] + r1 * M0[1] + r2 * M0[2] + (double)cam.T[2];
        const double Szz = r0 * (r0 * Sig[0] + r1 * Sig[1] + r2 * Sig[2]) +
                           r1 * (r0 * Sig[1] + r1 * Sig[3] + r2 * Sig[4]) +
                           r2 * (r0 * Sig[2] + r1 * Sig[4] + r2 * Sig[5]);
        const double zhi = Mz + sqrt(rad2 * Szz);
        if (zhi > 0.0) key = float_order_key(__double2float_rd(depth_bound(Mz, Szz, rad2, cam.F)));
    }
    keys[n] = key;
    vals[n] = (uint32_t)n;
}

__global__ void k_prep_records(const float* __restrict__ means, const float* __restrict__ covs, int N, CamDev cam,
                               double rad2, const uint32_t* __restrict__ skeys, const uint32_t* __restrict__ svals,
                               CullRec* __restrict__ cull, TraceRec* __restrict__ rec, GeoRec* __restrict__ geo) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    const uint32_t n = svals[r];
    TraceRec tr = {};
    tr.idx = n;
    tr.rank = (uint32_t)r;
    tr.tlo = INFINITY;
    CullRec cr;
    cr.i0 = 1; cr.i1 = 0; cr.j0 = 1; cr.j1 = 0;
    cr.tlo = INFINITY;
    cr.pad = 0;
    GeoRec g = {};
    if (skeys[r] != KEY_CULLED) {
        double M0[3], Sig[6], S0[6];
        load_kernel(means, covs, (int)n, M0, Sig);
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
        const float tlo = __double2float_rd(depth_bound(M[2], Sc[5], rad2, F));
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
        }
    }
    cull[r] = cr;
    rec[r] = tr;
    geo[r] = g;
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

// exclusive scan of n counters, one block of 1024 threads: each thread scans
// a contiguous run serially, then the run totals are scanned in LDS
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t* __restrict__ hist, int n) {
    __shared__ uint32_t buf[1024];
    const int tid = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int b0 = tid * per;
    uint32_t run = 0;
    for (int j = 0; j < per; ++j)
        if (b0 + j < n) run += hist[b0 + j];
    buf[tid] = run;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t y = tid >= off ? buf[tid - off] : 0u;
        __syncthreads();
        buf[tid] += y;
        __syncthreads();
    }
    uint32_t base = buf[tid] - run;
    for (int j = 0; j < per; ++j) {
        if (b0 + j < n) {
            const uint32_t x = hist[b0 + j];
            hist[b0 + j] = base;
            base += x;
        }
    }
}

__global__ __launch_bounds__(SORT_THREADS) void k_sort_scatter(const uint32_t* __restrict__ kin,
                                                                const uint32_t* __restrict__ vin,
                                                                uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                                int N, int shift, const uint32_t* __restrict__ hist,
                                                                int nblk) {
    __shared__ uint32_t offs[256];
    __shared__ uint32_t wcnt[SORT_THREADS / WAVE][256];
    const int tid = threadIdx.x, wave = tid / WAVE, lane = tid % WAVE;
    offs[tid] = hist[(size_t)tid * nblk + blockIdx.x];
    const int base = blockIdx.x * SORT_TILE;
    const uint64_t lt = lanemask_lt();
    (void)lane;
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

__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t n, uint32_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// zero three float ranges in one launch
__global__ void k_zero3(float* __restrict__ a, size_t na, float* __restrict__ b, size_t nb, float* __restrict__ c,
                        size_t nc) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < na) { a[i] = 0.f; return; }
    i -= na;
    if (i < nb) { b[i] = 0.f; return; }
    i -= nb;
    if (i < nc) c[i] = 0.f;
}

// ------------------------------------------------------------- launchers
void launch_zero3(float* a, size_t na, float* b, size_t nb, float* c, size_t nc, hipStream_t s) {
    const size_t n = na + nb + nc;
    if (n == 0) return;
    hipLaunchKernelGGL(k_zero3, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, na, b, nb, c, nc);
}

void launch_fill_u32(void* p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return;
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, n, v);
}

void launch_prep(const float* means, const float* covs, int N, const CamDev& cam, double rad2, const WsPtrs& w,
                 hipStream_t s) {
    if (N <= 0) return;
    const int blocks = (N + 255) / 256;
    hipLaunchKernelGGL(k_prep_keys, dim3(blocks), dim3(256), 0, s, means, covs, N, cam, rad2, w.keys, w.vals,
                       &w.hdr->status);
    // four stable 8-bit passes: keys/vals -> keys2/vals2 -> keys/vals -> ...
    const int nblk = sort_blocks(N);
    uint32_t* kin = w.keys;
    uint32_t* vin = w.vals;
    uint32_t* kout = w.keys2;
    uint32_t* vout = w.vals2;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_sort_hist, dim3(nblk), dim3(SORT_THREADS), 0, s, kin, N, shift, w.hist, nblk);
        hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, w.hist, nblk * 256);
        hipLaunchKernelGGL(k_sort_scatter, dim3(nblk), dim3(SORT_THREADS), 0, s, kin, vin, kout, vout, N, shift,
                           w.hist, nblk);
        uint32_t* t = kin; kin = kout; kout = t;
        t = vin; vin = vout; vout = t;
    }
    hipLaunchKernelGGL(k_prep_records, dim3(blocks), dim3(256), 0, s, means, covs, N, cam, rad2, kin, vin, w.cull,
                       w.rec, w.geo);
}

}  // namespace voge
