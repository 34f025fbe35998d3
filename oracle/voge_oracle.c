/*
 * voge_oracle.c -- FP64 CPU oracle for the VoGE rendering equations.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * tests and the benchmark's CPU-baseline leg use to check and time the GPU
 * library.  It shares no code, header, table or helper with the GPU path and
 * must never be called by it.
 *
 * Every step follows "VoGE: A Differentiable Volume Renderer using Gaussian
 * Ellipsoids for Analysis-by-Synthesis" (Wang et al., ICLR 2023):
 *   - viewing transform of centres and inverse covariances (Sec. 3.3, Eq. 3-4)
 *   - perspective rays (Sec. 3.3, Eq. 5)
 *   - ray tracing: l, q and 1/sigma^2 per kernel (Sec. 3.3, Eq. 6; App. A.1)
 *   - fine selection: keep kernels with e^q > eta, sort by l, take the K'
 *     nearest (Sec. 3.3 "Coarse-to-fine rendering"; App. A.3)
 *   - transmittance as an erf sum (Eq. 7; App. A.2) and the closed-form colour
 *     C = sum_k T(l_k) e^{q_k} c_k (Eq. 8; App. A.2)
 *   - analytic gradients of that closed form (the paper states the renderer is
 *     differentiable w.r.t. camera and ellipsoids, Sec. 3.3, and that both the
 *     T(l_k) and e^{q_k} paths carry gradient, App. C ablation)
 *   - the exact outer integral of Eq. 1 for the same kept set, by quadrature
 *     (the comparison of Fig. "approximate", App. A.2), used only to bound the
 *     approximation error.
 *
 * Readings where the paper is silent or inconsistent:
 *   tau = 1; the along-ray mass of kernel m is e^{q_m} (the normalisation
 *   1/sqrt(2 pi ||Sigma||) is dropped, as in App. A.2); the erf argument is
 *   (t - l_m) * sqrt(a_m) with a_m = D^T S_m D, exactly as printed; the
 *   transmittance sum runs over the kept set including k itself; ties in l are
 *   broken by kernel index; a kernel must also have l > 0; S = R S0 R^T
 *   (column-vector convention of Eq. 3); D has unit z (Eq. 5); pixel (i, j)
 *   is row i, column j at integer coordinates; background is 0; a covariance
 *   that is not symmetric positive definite is skipped and counted.
 *
 * Precision: all arithmetic and all inputs in double (callers widen float32
 * inputs exactly).  Parallelism: OpenMP over pixels only (no blocking or reordering
 * of the arithmetic).
 */
#define _USE_MATH_DEFINES
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define OR_FLAG_TIE 1      /* |l_K - l_{K+1}| <= 1e-6 l_K: the K-th place is a near tie   */
#define OR_FLAG_ETA 2      /* some kernel with l > 0 sits within 1e-5 of the threshold q  */

/* Noise-floor mode of oracle_backward (jitter != 0): every per-pair
 * derivative -- dL/dq, dL/dl and dL/da of a (pixel, kept kernel) pair and its
 * weight W in the attribute gradient -- is multiplied by 1 + s 2^-24 with a
 * sign s = +-1 drawn per (seed, pixel, kernel, quantity), i.e. moved by the
 * unit roundoff of FP32, as an implementation that carries those quantities
 * in FP32 rounds them.  The signs come from SplitMix64 (Steele, Lea and Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014), a counter
 * hash, so a draw does not depend on threads or order.  A diagnostic of the
 * spread no FP32 implementation can beat; the default (jitter = 0) is the
 * plain FP64 backward. */
static double pair_jitter(uint64_t seed, int64_t pixel, int kernel, int which) {
    uint64_t z = seed ^ ((uint64_t)pixel * 0x100000001B3ull) ^ ((uint64_t)kernel << 3) ^ (uint64_t)which;
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (z >> 63) ? 1.0 + ldexp(1.0, -24) : 1.0 - ldexp(1.0, -24);
}

/* gradient ablations of oracle_backward (grad_mode bits) */
#define ORACLE_BLOCK_T 1     /* no gradient through the transmittance T(l_k)               */
#define ORACLE_BLOCK_RHO 2   /* no gradient through the factor e^{q_k} of Eq. 8            */

typedef struct {
    double R[9], T[3];
    double F, Ox, Oy;
    int H, W;
} cam_t;

typedef struct {
    double M0[3];   /* centre, object space                         */
    double S0[9];   /* inverse covariance, object space             */
    double M[3];    /* centre, camera space (Eq. 3)                 */
    double S[9];    /* inverse covariance, camera space (Eq. 4)     */
    int valid;
} ker_t;

typedef struct {
    double l, q, a;
    int idx;
} cand_t;

/* ---------------------------------------------------------------------- */
/* small dense helpers (3x3, row-major)                                    */
/* ---------------------------------------------------------------------- */

static void mat_vec(const double A[9], const double x[3], double y[3]) {
    for (int r = 0; r < 3; ++r) y[r] = A[3 * r] * x[0] + A[3 * r + 1] * x[1] + A[3 * r + 2] * x[2];
}

static void mat_t_vec(const double A[9], const double x[3], double y[3]) {
    for (int r = 0; r < 3; ++r) y[r] = A[r] * x[0] + A[3 + r] * x[1] + A[6 + r] * x[2];
}

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void mat_mul(const double A[9], const double B[9], double C[9]) {
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}

static void mat_transpose(const double A[9], double B[9]) {
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) B[3 * c + r] = A[3 * r + c];
}

/* Inverse of a symmetric positive-definite 3x3 matrix through its Cholesky
 * factor.  Returns 0 when A is not SPD or not finite. */
static int spd_inverse(const double A[9], double Ainv[9]) {
    double L[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < 9; ++i)
        if (!isfinite(A[i])) return 0;
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[3 * i + j];
            for (int k = 0; k < j; ++k) s -= L[3 * i + k] * L[3 * j + k];
            if (i == j) {
                if (!(s > 0.0)) return 0;
                L[3 * i + i] = sqrt(s);
            } else {
                L[3 * i + j] = s / L[3 * j + j];
            }
        }
    }
    for (int col = 0; col < 3; ++col) {
        double y[3], x[3];
        for (int i = 0; i < 3; ++i) {            /* L y = e_col */
            double s = (i == col) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) s -= L[3 * i + k] * y[k];
            y[i] = s / L[3 * i + i];
        }
        for (int i = 2; i >= 0; --i) {           /* L^T x = y */
            double s = y[i];
            for (int k = i + 1; k < 3; ++k) s -= L[3 * k + i] * x[k];
            x[i] = s / L[3 * i + i];
        }
        for (int i = 0; i < 3; ++i) Ainv[3 * i + col] = x[i];
    }
    for (int i = 0; i < 9; ++i)
        if (!isfinite(Ainv[i])) return 0;
    return 1;
}

static void load_camera(const double* cam15, int H, int W, cam_t* cam) {
    for (int i = 0; i < 9; ++i) cam->R[i] = (double)cam15[i];
    for (int i = 0; i < 3; ++i) cam->T[i] = (double)cam15[9 + i];
    cam->F = (double)cam15[12];
    cam->Ox = (double)cam15[13];
    cam->Oy = (double)cam15[14];
    cam->H = H;
    cam->W = W;
}

/* ---------------------------------------------------------------------- */
/* Step 1: viewing transformation (Sec. 3.3, Eq. 3 and Eq. 4)              */
/*   M = R M0 + T;   S = Sigma^{-1} in camera space = R S0 R^T             */
/* ---------------------------------------------------------------------- */
static int prepare_kernels(const double* means, const double* covs, int N, const cam_t* cam, ker_t* ks) {
    int n_invalid = 0;
    double Rt[9];
    mat_transpose(cam->R, Rt);
    for (int n = 0; n < N; ++n) {
        ker_t* k = &ks[n];
        const double* c = covs + 6 * (size_t)n;
        double Sigma[9] = {c[0], c[1], c[2], c[1], c[3], c[4], c[2], c[4], c[5]};
        for (int d = 0; d < 3; ++d) k->M0[d] = means[3 * (size_t)n + d];
        k->valid = spd_inverse(Sigma, k->S0) && isfinite(k->M0[0]) && isfinite(k->M0[1]) && isfinite(k->M0[2]);
        if (!k->valid) {
            ++n_invalid;
            continue;
        }
        double RM[3];
        mat_vec(cam->R, k->M0, RM);
        for (int d = 0; d < 3; ++d) k->M[d] = RM[d] + cam->T[d];
        double tmp[9];
        mat_mul(cam->R, k->S0, tmp);
        mat_mul(tmp, Rt, k->S);
    }
    return n_invalid;
}

/* Step 2: perspective ray of pixel (i, j) (Sec. 3.3, Eq. 5). */
static void pixel_ray(const cam_t* cam, int i, int j, double D[3]) {
    D[0] = ((double)i - cam->Oy) / cam->F;
    D[1] = ((double)j - cam->Ox) / cam->F;
    D[2] = 1.0;
}

/* Step 3: ray tracing of one kernel (Sec. 3.3, Eq. 6; App. A.1):
 *   l = (M^T S D + D^T S M) / (2 D^T S D)   -- depth of the peak along the ray
 *   V = M - l D,  q = -1/2 V^T S V          -- log of the peak density
 *   a = 1/sigma^2 = D^T S D                 -- the 1D precision along the ray */
static void trace_kernel(const ker_t* k, const double D[3], double* l, double* q, double* a) {
    double SD[3], SM[3], V[3], SV[3];
    mat_vec(k->S, D, SD);
    mat_vec(k->S, k->M, SM);
    double dSd = dot3(D, SD);
    *l = (dot3(k->M, SD) + dot3(D, SM)) / (2.0 * dSd);
    for (int d = 0; d < 3; ++d) V[d] = k->M[d] - (*l) * D[d];
    mat_vec(k->S, V, SV);
    *q = -0.5 * dot3(V, SV);
    *a = dSd;
}

static int cand_cmp(const void* x, const void* y) {
    const cand_t* u = (const cand_t*)x;
    const cand_t* v = (const cand_t*)y;
    if (u->l < v->l) return -1;
    if (u->l > v->l) return 1;
    return (u->idx > v->idx) - (u->idx < v->idx);
}

/* Step 5 (Eq. 7; App. A.2): the optical depth
 *   E(t) = sum_m e^{q_m} (erf((t - l_m)/sigma_m) + 1) / 2,  sigma_m = a_m^{-1/2},
 * so that T(t) = exp(-tau E(t)) with tau = 1. */
static double optical_depth(double t, const cand_t* set, int n) {
    double E = 0.0;
    for (int m = 0; m < n; ++m)
        E += exp(set[m].q) * (erf((t - set[m].l) * sqrt(set[m].a)) + 1.0) / 2.0;
    return E;
}

/* Steps 3-4 for one pixel: trace every kernel, keep those with e^q > eta and
 * l > 0, sort by (l, index), keep the first K.  Returns K_eff; writes the
 * number of passing kernels and the near-tie / near-threshold flags. */
static int select_kernels(const ker_t* ks, int N, const int* list, const double D[3], double lneta, int K,
                          cand_t* scratch, int* n_pass_out, int* flags_out) {
    int n = 0, flags = 0;
    double near_l = INFINITY;   /* smallest l among kernels within 1e-5 of the threshold */
    for (int t = 0; t < N; ++t) {
        const int k = list ? list[t] : t;     /* every kernel, or a tile's candidates */
        if (!ks[k].valid) continue;
        double l, q, a;
        trace_kernel(&ks[k], D, &l, &q, &a);
        if (l > 0.0 && fabs(q - lneta) <= 1e-5 && l < near_l) near_l = l;
        if (q > lneta && l > 0.0) {
            scratch[n].l = l;
            scratch[n].q = q;
            scratch[n].a = a;
            scratch[n].idx = k;
            ++n;
        }
    }
    qsort(scratch, (size_t)n, sizeof(cand_t), cand_cmp);
    int keff = n < K ? n : K;
    if (n > K && (scratch[K].l - scratch[K - 1].l) <= 1e-6 * fabs(scratch[K - 1].l)) flags |= OR_FLAG_TIE;
    /* a near-threshold kernel matters only if it could enter or leave the kept set */
    double lmax = (keff == K && keff > 0) ? scratch[K - 1].l : INFINITY;
    if (isfinite(near_l) && near_l <= lmax * (1.0 + 1e-6)) flags |= OR_FLAG_ETA;
    *n_pass_out = n;
    *flags_out = flags;
    return keff;
}

/* Optional coarse stage for timing (the CPU baseline's binned mode): the
 * paper's coarse-to-fine rendering (Sec. 3.3; App. A.3) skips kernels that
 * cannot reach a pixel.  Here each kernel's candidates are the 16x16 screen
 * tiles met by the projection of a sphere around its centre that contains
 * every point where (X - M)^T S (X - M) <= 2 ln(1/eta) + 1e-4: radius^2 =
 * (2 ln(1/eta) + 1e-4) trace(Sigma), trace(Sigma) >= its largest
 * eigenvalue.  A kernel with q >= ln(eta) - 5e-5 at a pixel has its peak on
 * that pixel's ray inside the sphere, so no kernel that passes the
 * threshold or could set a flag is skipped, and the results equal the
 * brute-force ones bit for bit (the candidates keep ascending index order).
 * A sphere that reaches z <= 1e-9 covers the whole image. */
#define OR_BIN 16

typedef struct {
    int ntx, nty;
    int64_t* off;     /* [ntx*nty + 1] */
    int* idx;         /* kernel indices per tile, ascending */
} bins_t;

static void sphere_rows(double Mx, double Mz, double r, double F, double O, double* lo, double* hi) {
    /* tangent planes x = k z of the sphere: (Mx - k Mz)^2 = r^2 (1 + k^2) */
    const double a = Mz * Mz - r * r, d = sqrt(Mx * Mx + Mz * Mz - r * r);
    const double k1 = (Mx * Mz - r * d) / a, k2 = (Mx * Mz + r * d) / a;
    *lo = O + F * (k1 < k2 ? k1 : k2);
    *hi = O + F * (k1 < k2 ? k2 : k1);
}

static void build_bins(const ker_t* ks, const double* covs, int N, const cam_t* cam, double eta, bins_t* b) {
    const int H = cam->H, W = cam->W;
    b->ntx = (W + OR_BIN - 1) / OR_BIN;
    b->nty = (H + OR_BIN - 1) / OR_BIN;
    const int nt = b->ntx * b->nty;
    int* box = (int*)malloc(sizeof(int) * 4 * (size_t)(N > 0 ? N : 1));
    b->off = (int64_t*)calloc((size_t)nt + 1, sizeof(int64_t));
    const double grow = 2.0 * log(1.0 / eta) + 1e-4;
    for (int n = 0; n < N; ++n) {
        int* bx = box + 4 * n;
        bx[0] = 1; bx[1] = 0; bx[2] = 1; bx[3] = 0;           /* empty */
        if (!ks[n].valid) continue;
        const double* c = covs + 6 * (size_t)n;
        const double r = sqrt(grow * (c[0] + c[3] + c[5]));
        const double* M = ks[n].M;
        double i0 = 0, i1 = H - 1, j0 = 0, j1 = W - 1;
        if (M[2] - r > 1e-9) {
            double lo, hi;
            sphere_rows(M[0], M[2], r, cam->F, cam->Oy, &lo, &hi);
            i0 = fmax(i0, floor(lo) - 1.0);
            i1 = fmin(i1, ceil(hi) + 1.0);
            sphere_rows(M[1], M[2], r, cam->F, cam->Ox, &lo, &hi);
            j0 = fmax(j0, floor(lo) - 1.0);
            j1 = fmin(j1, ceil(hi) + 1.0);
        }
        if (i0 > i1 || j0 > j1) continue;
        bx[0] = (int)i0 / OR_BIN; bx[1] = (int)i1 / OR_BIN;
        bx[2] = (int)j0 / OR_BIN; bx[3] = (int)j1 / OR_BIN;
        for (int ti = bx[0]; ti <= bx[1]; ++ti)
            for (int tj = bx[2]; tj <= bx[3]; ++tj) b->off[ti * b->ntx + tj + 1] += 1;
    }
    for (int t = 0; t < nt; ++t) b->off[t + 1] += b->off[t];
    b->idx = (int*)malloc(sizeof(int) * (size_t)(b->off[nt] > 0 ? b->off[nt] : 1));
    int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nt > 0 ? nt : 1));
    for (int t = 0; t < nt; ++t) cur[t] = b->off[t];
    for (int n = 0; n < N; ++n) {                              /* ascending n in every tile */
        const int* bx = box + 4 * n;
        for (int ti = bx[0]; ti <= bx[1]; ++ti)
            for (int tj = bx[2]; tj <= bx[3]; ++tj) b->idx[cur[ti * b->ntx + tj]++] = n;
    }
    free(cur);
    free(box);
}

static void free_bins(bins_t* b) {
    free(b->off);
    free(b->idx);
}

/* Step 4 on every kernel, or (bins) on the candidates of the pixel's tile. */
static int select_pixel(const ker_t* ks, int N, const bins_t* bins, int i, int j, const double D[3],
                        double lneta, int K, cand_t* scratch, int* n_pass_out, int* flags_out) {
    if (!bins) return select_kernels(ks, N, NULL, D, lneta, K, scratch, n_pass_out, flags_out);
    const int t = (i / OR_BIN) * bins->ntx + j / OR_BIN;
    return select_kernels(ks, (int)(bins->off[t + 1] - bins->off[t]), bins->idx + bins->off[t], D, lneta, K,
                          scratch, n_pass_out, flags_out);
}

/* Step 4 replaced by a given kept set (the set another implementation
 * selected for this pixel): `row` holds up to K kernel indices, -1 padded.
 * Each listed kernel is traced as in step 3 and the set is put in (l, index)
 * order; nothing is filtered, so steps 5-6 and the backward then run on
 * exactly that set.  The caller has checked every index (see
 * check_given).  Returns the set's size. */
static int given_kernels(const ker_t* ks, const double D[3], const int32_t* row, int K, cand_t* out) {
    int n = 0;
    for (int s = 0; s < K; ++s) {
        if (row[s] < 0) continue;
        double l, q, a;
        trace_kernel(&ks[row[s]], D, &l, &q, &a);
        out[n].l = l;
        out[n].q = q;
        out[n].a = a;
        out[n].idx = row[s];
        ++n;
    }
    qsort(out, (size_t)n, sizeof(cand_t), cand_cmp);
    return n;
}

/* A given kept set may only name valid kernels, each at most once per pixel. */
static int check_given(const ker_t* ks, int N, const int32_t* given, int64_t npx, int K) {
    for (int64_t p = 0; p < npx; ++p) {
        const int32_t* row = given + p * K;
        for (int s = 0; s < K; ++s) {
            if (row[s] < 0) continue;
            if (row[s] >= N || !ks[row[s]].valid) return -1;
            for (int t = 0; t < s; ++t)
                if (row[t] == row[s]) return -1;
        }
    }
    return 0;
}

/* Steps 5-6 (Eq. 7-8): T_k = exp(-E(l_k)), W_k = T_k e^{q_k}. */
static void blend_weights(const cand_t* kept, int keff, double* E, double* Wt) {
    for (int k = 0; k < keff; ++k) {
        E[k] = optical_depth(kept[k].l, kept, keff);
        Wt[k] = exp(-E[k]) * exp(kept[k].q);
    }
}

static int check_args(int N, int C, int H, int W, double eta, int K) {
    if (N < 0 || C < 1 || H < 1 || W < 1 || K < 1) return -1;
    if (!(eta > 0.0 && eta < 1.0)) return -1;
    return 0;
}

static int nthreads_of(int req) {
#ifdef _OPENMP
    return req > 0 ? req : omp_get_max_threads();
#else
    (void)req;
    return 1;
#endif
}

/* ====================================================================== */
/* Public entry points (ctypes)                                            */
/* ====================================================================== */

/* Forward render of the pixels in `pix` (linear index i*W + j; NULL = all).
 * Outputs (any may be NULL):
 *   image[n_pix*C]   C_p = sum_k W_k c_k                              (Eq. 8)
 *   wsum[n_pix]      sum_k W_k
 *   absum[n_pix*C]   sum_k W_k |c_k|  (the scale of each image element)
 *   kept_idx[n_pix*K]     kernel indices of the kept set, -1 padded
 *   kept_rec[n_pix*K*5]   (l, q, a, E(l_k), W_k) of each kept entry
 *   n_pass[n_pix]    number of kernels with e^q > eta and l > 0
 *   flags[n_pix]     OR_FLAG_TIE | OR_FLAG_ETA
 * given[n_pix*K] (optional): kept sets chosen elsewhere (-1 padded).  Step 4
 * is then skipped and steps 5-6 run on exactly these sets (n_pass = -1,
 * flags = 0); an index out of range, of a skipped kernel or repeated within
 * a pixel is a bad argument.
 * binned: take step 4's candidates from 16x16 screen tiles (see build_bins;
 * same results, less work; a timing mode of the CPU baseline).
 * Returns the number of skipped (non-SPD / non-finite) kernels, or -1 on bad
 * arguments. */
int oracle_forward(const double* means, const double* covs, const double* attrs, int N, int C,
                   const double* cam15, int H, int W, double eta, int K,
                   const int64_t* pix, int64_t n_pix, int nthreads,
                   double* image, double* wsum, double* absum, int32_t* kept_idx, double* kept_rec,
                   int32_t* n_pass, int32_t* flags, const int32_t* given, int binned) {
    if (check_args(N, C, H, W, eta, K)) return -1;
    cam_t cam;
    load_camera(cam15, H, W, &cam);
    ker_t* ks = (ker_t*)calloc((size_t)(N > 0 ? N : 1), sizeof(ker_t));
    int n_invalid = prepare_kernels(means, covs, N, &cam, ks);
    const double lneta = log(eta);
    const int64_t npx = pix ? n_pix : (int64_t)H * W;
    if (given && check_given(ks, N, given, npx, K)) {
        free(ks);
        return -1;
    }
    bins_t bins;
    if (binned && !given) build_bins(ks, covs, N, &cam, eta, &bins);
    const bins_t* bp = (binned && !given) ? &bins : NULL;

#pragma omp parallel num_threads(nthreads_of(nthreads))
    {
        cand_t* scratch = (cand_t*)malloc(sizeof(cand_t) * (size_t)(N > 0 ? N : 1));
        double* E = (double*)malloc(sizeof(double) * (size_t)K);
        double* Wt = (double*)malloc(sizeof(double) * (size_t)K);
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npx; ++p) {
            int64_t lin = pix ? pix[p] : p;
            int i = (int)(lin / W), j = (int)(lin % W);
            double D[3];
            pixel_ray(&cam, i, j, D);
            int np_ = -1, fl = 0;
            int keff = given ? given_kernels(ks, D, given + p * K, K, scratch)
                             : select_pixel(ks, N, bp, i, j, D, lneta, K, scratch, &np_, &fl);
            blend_weights(scratch, keff, E, Wt);
            double ws = 0.0;
            for (int k = 0; k < keff; ++k) ws += Wt[k];
            for (int c = 0; c < C; ++c) {
                double acc = 0.0, aacc = 0.0;
                for (int k = 0; k < keff; ++k) {
                    double ck = (double)attrs[(size_t)scratch[k].idx * C + c];
                    acc += Wt[k] * ck;
                    aacc += Wt[k] * fabs(ck);
                }
                if (image) image[p * C + c] = acc;
                if (absum) absum[p * C + c] = aacc;
            }
            if (wsum) wsum[p] = ws;
            if (n_pass) n_pass[p] = np_;
            if (flags) flags[p] = fl;
            for (int k = 0; k < K; ++k) {
                if (kept_idx) kept_idx[p * K + k] = k < keff ? scratch[k].idx : -1;
                if (kept_rec) {
                    double* r = kept_rec + (p * K + k) * 5;
                    if (k < keff) {
                        r[0] = scratch[k].l;
                        r[1] = scratch[k].q;
                        r[2] = scratch[k].a;
                        r[3] = E[k];
                        r[4] = Wt[k];
                    } else {
                        r[0] = r[1] = r[2] = r[3] = r[4] = 0.0;
                    }
                }
            }
        }
        free(scratch);
        free(E);
        free(Wt);
    }
    if (bp) free_bins(&bins);
    free(ks);
    return n_invalid;
}

/* T(t) = exp(-E(t)) for an explicit set of (l, q, a) records (Eq. 7), the same
 * function the forward evaluates at t = l_k.  rec is n x 3 (l, q, a). */
void oracle_transmittance(const double* rec, int n, const double* t, int nt, double* T_out) {
    cand_t* set = (cand_t*)malloc(sizeof(cand_t) * (size_t)(n > 0 ? n : 1));
    for (int m = 0; m < n; ++m) {
        set[m].l = rec[3 * m];
        set[m].q = rec[3 * m + 1];
        set[m].a = rec[3 * m + 2];
        set[m].idx = m;
    }
    for (int s = 0; s < nt; ++s) T_out[s] = exp(-optical_depth(t[s], set, n));
    free(set);
}

/* Backward of the forward above for the pixels in `pix` with upstream
 * gradient grad_pix[n_pix*C] (the rest of the image has zero gradient).  The
 * kept set of each pixel is held fixed.  Gradients (all overwritten):
 *   g_means[N*3], g_covs[N*6] (w.r.t. the 6 packed numbers, off-diagonals once),
 *   g_attrs[N*C], g_cam[15] (R row-major, T, F, O_x, O_y).
 * a_* (optional) receive, per element, the scale for comparisons: every
 * term of the computation carried with its absolute value through the same
 * linear steps (each pair term of the transmittance derivative, each term of
 * the chain to world space), i.e. the sum of the absolute values of all
 * per-pair contributions to that element.
 * grad_mode: 0, or ORACLE_BLOCK_T and/or ORACLE_BLOCK_RHO (the gradient
 * ablations of the paper's pose-estimation ablation table).
 * given (optional): kept sets chosen elsewhere, as for oracle_forward; the
 * gradients are then those of the forward on exactly these sets.
 * binned: step 4 on the candidates of 16x16 screen tiles, as for
 * oracle_forward.
 * Returns the number of skipped kernels or -1. */
int oracle_backward(const double* means, const double* covs, const double* attrs, int N, int C,
                    const double* cam15, int H, int W, double eta, int K,
                    const int64_t* pix, int64_t n_pix, const double* grad_pix, int nthreads,
                    double* g_means, double* g_covs, double* g_attrs, double* g_cam,
                    double* a_means, double* a_covs, double* a_attrs, double* a_cam, int grad_mode,
                    const int32_t* given, int binned, uint64_t jitter) {
    if (check_args(N, C, H, W, eta, K)) return -1;
    cam_t cam;
    load_camera(cam15, H, W, &cam);
    ker_t* ks = (ker_t*)calloc((size_t)(N > 0 ? N : 1), sizeof(ker_t));
    int n_invalid = prepare_kernels(means, covs, N, &cam, ks);
    const double lneta = log(eta);
    const int64_t npx = pix ? n_pix : (int64_t)H * W;
    if (given && check_given(ks, N, given, npx, K)) {
        free(ks);
        return -1;
    }
    bins_t bins;
    if (binned && !given) build_bins(ks, covs, N, &cam, eta, &bins);
    const bins_t* bp = (binned && !given) ? &bins : NULL;
    const int nt = nthreads_of(nthreads);
    const size_t per = (size_t)N * (3 + 6 + (size_t)C) + 15;   /* one thread's accumulators */
    double* acc = (double*)calloc(per * (size_t)nt * 2, sizeof(double));
    double Rt[9];
    mat_transpose(cam.R, Rt);

#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* gM = acc + per * (size_t)tid * 2;         /* N*3 world-space centre grads  */
        double* gC = gM + (size_t)N * 3;                   /* N*6 packed covariance grads   */
        double* gA = gC + (size_t)N * 6;                   /* N*C attribute grads           */
        double* gK = gA + (size_t)N * C;                   /* 15 camera grads               */
        double* aM = gM + per;                             /* absolute-contribution sums    */
        double* aC = aM + (size_t)N * 3;
        double* aA = aC + (size_t)N * 6;
        double* aK = aA + (size_t)N * C;
        cand_t* kept = (cand_t*)malloc(sizeof(cand_t) * (size_t)(N > 0 ? N : 1));
        double* E = (double*)malloc(sizeof(double) * (size_t)K);
        double* Wt = (double*)malloc(sizeof(double) * (size_t)K);
        double* dm = (double*)malloc(sizeof(double) * (size_t)K * 8);
        double* dl = dm + K;
        double* da = dl + K;
        double* dE = da + K;
        double* adm = dE + K;      /* absolute-value companions of dm, dl, da, dE */
        double* adl = adm + K;
        double* ada = adl + K;
        double* adE = ada + K;

#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npx; ++p) {
            int64_t lin = pix ? pix[p] : p;
            int i = (int)(lin / W), j = (int)(lin % W);
            const double* G = grad_pix + p * C;
            double D[3];
            pixel_ray(&cam, i, j, D);
            int np_, fl;
            int keff = given ? given_kernels(ks, D, given + p * K, K, kept)
                             : select_pixel(ks, N, bp, i, j, D, lneta, K, kept, &np_, &fl);
            if (keff == 0) continue;
            blend_weights(kept, keff, E, Wt);
            /* C = sum_k W_k c_k:  dL/dc_k = W_k G;  dL/dW_k = G . c_k */
            for (int k = 0; k < keff; ++k) {
                const double* ck = attrs + (size_t)kept[k].idx * C;
                double g = 0.0, ag = 0.0;
                const double wj = jitter ? Wt[k] * pair_jitter(jitter, lin, kept[k].idx, 3) : Wt[k];
                for (int c = 0; c < C; ++c) {
                    g += G[c] * ck[c];
                    ag += fabs(G[c] * ck[c]);
                    gA[(size_t)kept[k].idx * C + c] += wj * G[c];
                    aA[(size_t)kept[k].idx * C + c] += fabs(Wt[k] * G[c]);
                }
                /* W_k = exp(-E_k) e^{q_k}: direct path through e^{q_k}, and dL/dE_k.
                 * The ablations of the paper's pose-estimation table stop one
                 * of the two: ORACLE_BLOCK_T the path through the
                 * transmittance T = exp(-E), ORACLE_BLOCK_RHO the direct
                 * factor e^{q_k} of Eq. 8 (e^{q_m} inside E stays). */
                dm[k] = (grad_mode & ORACLE_BLOCK_RHO) ? 0.0 : g * exp(-E[k]);
                adm[k] = (grad_mode & ORACLE_BLOCK_RHO) ? 0.0 : ag * exp(-E[k]);
                dE[k] = (grad_mode & ORACLE_BLOCK_T) ? 0.0 : -g * Wt[k];
                adE[k] = (grad_mode & ORACLE_BLOCK_T) ? 0.0 : ag * Wt[k];
                dl[k] = da[k] = adl[k] = ada[k] = 0.0;
            }
            /* E_k = sum_m m_m Phi(x_km),  x_km = (l_k - l_m) sqrt(a_m),
             * Phi(x) = (1 + erf x)/2,  Phi'(x) = exp(-x^2)/sqrt(pi) */
            for (int k = 0; k < keff; ++k) {
                for (int m = 0; m < keff; ++m) {
                    double s_m = sqrt(kept[m].a);
                    double x = (kept[k].l - kept[m].l) * s_m;
                    double Phi = (1.0 + erf(x)) / 2.0;
                    double dPhi = exp(-x * x) / sqrt(M_PI);
                    double mm = exp(kept[m].q);
                    dm[m] += dE[k] * Phi;
                    adm[m] += adE[k] * Phi;
                    double dx = dE[k] * mm * dPhi;
                    double adx = adE[k] * mm * dPhi;
                    dl[k] += dx * s_m;
                    dl[m] -= dx * s_m;
                    adl[k] += adx * s_m;
                    adl[m] += adx * s_m;
                    da[m] += dx * (kept[k].l - kept[m].l) / (2.0 * s_m);
                    ada[m] += adx * fabs(kept[k].l - kept[m].l) / (2.0 * s_m);
                }
            }
            /* chain (q, l, a) -> camera-space (M, S) and the ray D (App. A.1):
             *   dq/dM = -S V,  dq/dS = -V V^T/2,  dq/dD = l S V
             *   dl/dM = S D/a, dl/dS = D V^T/a,   dl/dD = (S V - l S D)/a
             *   da/dS = D D^T,                    da/dD = 2 S D            */
            for (int k = 0; k < keff; ++k) {
                const ker_t* kk = &ks[kept[k].idx];
                double l = kept[k].l, a = kept[k].a;
                double dq = dm[k] * exp(kept[k].q);
                double adq = adm[k] * exp(kept[k].q);
                if (jitter) {
                    dq *= pair_jitter(jitter, lin, kept[k].idx, 0);
                    dl[k] *= pair_jitter(jitter, lin, kept[k].idx, 1);
                    da[k] *= pair_jitter(jitter, lin, kept[k].idx, 2);
                }
                double V[3], SV[3], SD[3];
                for (int d = 0; d < 3; ++d) V[d] = kk->M[d] - l * D[d];
                mat_vec(kk->S, V, SV);
                mat_vec(kk->S, D, SD);
                double gMc[3], GS[9], gD[3], agMc[3], aGS[9], agD[3];
                for (int d = 0; d < 3; ++d) {
                    gMc[d] = -dq * SV[d] + dl[k] * SD[d] / a;
                    agMc[d] = adq * fabs(SV[d]) + adl[k] * fabs(SD[d]) / a;
                    gD[d] = dq * l * SV[d] + dl[k] * (SV[d] - l * SD[d]) / a + da[k] * 2.0 * SD[d];
                    agD[d] = adq * l * fabs(SV[d]) + adl[k] * (fabs(SV[d]) + l * fabs(SD[d])) / a +
                             ada[k] * 2.0 * fabs(SD[d]);
                }
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) {
                        GS[3 * r + c] = -0.5 * dq * V[r] * V[c] + dl[k] * D[r] * V[c] / a + da[k] * D[r] * D[c];
                        aGS[3 * r + c] = 0.5 * adq * fabs(V[r] * V[c]) + adl[k] * fabs(D[r] * V[c]) / a +
                                         ada[k] * fabs(D[r] * D[c]);
                    }
                /* camera space -> world space (Eq. 3-4) */
                double aR[9], aS0[9], aM0[3];
                for (int e = 0; e < 9; ++e) {
                    aR[e] = fabs(cam.R[e]);
                    aS0[e] = fabs(kk->S0[e]);
                }
                for (int d = 0; d < 3; ++d) aM0[d] = fabs(kk->M0[d]);
                double aRt[9];
                mat_transpose(aR, aRt);
                double gMw[3], agMw[3];
                mat_t_vec(cam.R, gMc, gMw);                        /* R^T gM           */
                mat_t_vec(aR, agMc, agMw);
                double t1[9], GS0[9], t2[9], GSig[9];
                mat_mul(Rt, GS, t1);
                mat_mul(t1, cam.R, GS0);                           /* R^T G_S R        */
                mat_mul(kk->S0, GS0, t2);
                mat_mul(t2, kk->S0, GSig);                         /* S0 G S0          */
                for (int e = 0; e < 9; ++e) GSig[e] = -GSig[e];    /* d(A^-1) = -A^-1 dA A^-1 */
                double u1[9], aGS0[9], u2[9], aGSig[9];
                mat_mul(aRt, aGS, u1);
                mat_mul(u1, aR, aGS0);
                mat_mul(aS0, aGS0, u2);
                mat_mul(u2, aS0, aGSig);
                double pk[6] = {GSig[0], GSig[1] + GSig[3], GSig[2] + GSig[6],
                                GSig[4], GSig[5] + GSig[7], GSig[8]};
                double apk[6] = {aGSig[0], aGSig[1] + aGSig[3], aGSig[2] + aGSig[6],
                                 aGSig[4], aGSig[5] + aGSig[7], aGSig[8]};
                size_t n = (size_t)kept[k].idx;
                for (int d = 0; d < 3; ++d) {
                    gM[n * 3 + d] += gMw[d];
                    aM[n * 3 + d] += agMw[d];
                }
                for (int e = 0; e < 6; ++e) {
                    gC[n * 6 + e] += pk[e];
                    aC[n * 6 + e] += apk[e];
                }
                /* camera extrinsics: dL/dR = gM M0^T + G_S R S0^T + G_S^T R S0, dL/dT = gM */
                double gR[9], RS0[9], A1[9], A2[9], GSt[9];
                mat_mul(cam.R, kk->S0, RS0);
                mat_mul(GS, RS0, A1);          /* S0 symmetric: R S0^T = R S0 */
                mat_transpose(GS, GSt);
                mat_mul(GSt, RS0, A2);
                double aRS0[9], aA1[9], aA2[9], aGSt[9];
                mat_mul(aR, aS0, aRS0);
                mat_mul(aGS, aRS0, aA1);
                mat_transpose(aGS, aGSt);
                mat_mul(aGSt, aRS0, aA2);
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) {
                        gR[3 * r + c] = gMc[r] * kk->M0[c] + A1[3 * r + c] + A2[3 * r + c];
                        aK[3 * r + c] += agMc[r] * aM0[c] + aA1[3 * r + c] + aA2[3 * r + c];
                    }
                for (int e = 0; e < 9; ++e) gK[e] += gR[e];
                for (int d = 0; d < 3; ++d) {
                    gK[9 + d] += gMc[d];
                    aK[9 + d] += agMc[d];
                }
                /* intrinsics through D = ((i - O_y)/F, (j - O_x)/F, 1) (Eq. 5) */
                double F2 = cam.F * cam.F;
                double gF = -gD[0] * ((double)i - cam.Oy) / F2 - gD[1] * ((double)j - cam.Ox) / F2;
                double aF = agD[0] * fabs((double)i - cam.Oy) / F2 + agD[1] * fabs((double)j - cam.Ox) / F2;
                gK[12] += gF;
                gK[13] += -gD[1] / cam.F;
                gK[14] += -gD[0] / cam.F;
                aK[12] += aF;
                aK[13] += agD[1] / cam.F;
                aK[14] += agD[0] / cam.F;
            }
        }
        free(kept);
        free(E);
        free(Wt);
        free(dm);
    }
    /* reduce the per-thread accumulators in thread order */
    double* out_g[4] = {g_means, g_covs, g_attrs, g_cam};
    double* out_a[4] = {a_means, a_covs, a_attrs, a_cam};
    size_t off[4] = {0, (size_t)N * 3, (size_t)N * 9, (size_t)N * (9 + (size_t)C)};
    size_t len[4] = {(size_t)N * 3, (size_t)N * 6, (size_t)N * C, 15};
    for (int b = 0; b < 4; ++b) {
        for (size_t e = 0; e < len[b]; ++e) {
            double sg = 0.0, sa = 0.0;
            for (int t = 0; t < nt; ++t) {
                sg += acc[per * (size_t)t * 2 + off[b] + e];
                sa += acc[per * (size_t)t * 2 + per + off[b] + e];
            }
            if (out_g[b]) out_g[b][e] = sg;
            if (out_a[b]) out_a[b][e] = sa;
        }
    }
    if (bp) free_bins(&bins);
    free(acc);
    free(ks);
    return n_invalid;
}

/* The exact outer integral of Eq. 1 for the kept set of each pixel in `pix`,
 * with the along-ray density of kernel m taken as e^{q_m} g_m(t),
 *   g_m(t) = sqrt(a_m/pi) exp(-a_m (t - l_m)^2),
 * which is the density whose running integral is the erf sum of Eq. 7.  The
 * transmittance is exp(-E(t)) and the outer integral is a trapezoid rule on
 * n_samples points over [min_m l_m - 9/sqrt(a_m), max_m l_m + 9/sqrt(a_m)].
 * Outputs: w_exact[n_pix*K] and w_approx[n_pix*K] (the closed form, Eq. 8),
 * 0 padded; total[n_pix*2] = (sum_k w_exact, 1 - exp(-sum_m e^{q_m})). */
int oracle_quadrature(const double* means, const double* covs, int N, const double* cam15, int H, int W,
                      double eta, int K, const int64_t* pix, int64_t n_pix, int n_samples, int nthreads,
                      double* w_exact, double* w_approx, double* total) {
    if (check_args(N, 1, H, W, eta, K) || n_samples < 3) return -1;
    cam_t cam;
    load_camera(cam15, H, W, &cam);
    ker_t* ks = (ker_t*)calloc((size_t)(N > 0 ? N : 1), sizeof(ker_t));
    int n_invalid = prepare_kernels(means, covs, N, &cam, ks);
    const double lneta = log(eta);
    const int64_t npx = pix ? n_pix : (int64_t)H * W;
#pragma omp parallel num_threads(nthreads_of(nthreads))
    {
        cand_t* kept = (cand_t*)malloc(sizeof(cand_t) * (size_t)(N > 0 ? N : 1));
        double* E = (double*)malloc(sizeof(double) * (size_t)K);
        double* Wt = (double*)malloc(sizeof(double) * (size_t)K);
        double* acc = (double*)malloc(sizeof(double) * (size_t)K);
#pragma omp for schedule(dynamic, 4)
        for (int64_t p = 0; p < npx; ++p) {
            int64_t lin = pix ? pix[p] : p;
            int i = (int)(lin / W), j = (int)(lin % W);
            double D[3];
            pixel_ray(&cam, i, j, D);
            int np_, fl;
            int keff = select_kernels(ks, N, NULL, D, lneta, K, kept, &np_, &fl);
            blend_weights(kept, keff, E, Wt);
            double t0 = INFINITY, t1 = -INFINITY, msum = 0.0;
            for (int m = 0; m < keff; ++m) {
                double w = 9.0 / sqrt(kept[m].a);
                if (kept[m].l - w < t0) t0 = kept[m].l - w;
                if (kept[m].l + w > t1) t1 = kept[m].l + w;
                msum += exp(kept[m].q);
                acc[m] = 0.0;
            }
            if (keff > 0) {
                double h = (t1 - t0) / (double)(n_samples - 1);
                for (int s = 0; s < n_samples; ++s) {
                    double t = t0 + h * (double)s;
                    double wgt = (s == 0 || s == n_samples - 1) ? 0.5 * h : h;
                    double T = exp(-optical_depth(t, kept, keff));
                    for (int m = 0; m < keff; ++m) {
                        double g = sqrt(kept[m].a / M_PI) * exp(-kept[m].a * (t - kept[m].l) * (t - kept[m].l));
                        acc[m] += wgt * T * exp(kept[m].q) * g;
                    }
                }
            }
            double sum_exact = 0.0;
            for (int k = 0; k < K; ++k) {
                w_exact[p * K + k] = k < keff ? acc[k] : 0.0;
                w_approx[p * K + k] = k < keff ? Wt[k] : 0.0;
                if (k < keff) sum_exact += acc[k];
            }
            total[2 * p] = sum_exact;
            total[2 * p + 1] = 1.0 - exp(-msum);
        }
        free(kept);
        free(E);
        free(Wt);
        free(acc);
    }
    free(ks);
    return n_invalid;
}
