// epilogue.hip -- per-kernel epilogues.  Backward (FP64): camera-space
// gradients of each kernel back to world space, and the camera gradient.
// Sampler: the quotient of Eq. 10.
//
// With M = R M0 + T and S = R S0 R^T, S0 = Sigma^-1 (VoGE Sec. 3.3, Eq. 3-4),
// and G = the symmetric gradient w.r.t. S:
//   dL/dM0 = R^T dL/dM,   dL/dS0 = R^T G R,   dL/dSigma = -S0 (R^T G R) S0,
//   dL/dT = sum_k dL/dM_k,   dL/dR = sum_k [dL/dM_k M0_k^T + 2 G_k R S0_k].
// The covariance gradient is w.r.t. the 6 packed numbers, so each
// off-diagonal entry collects both of its matrix positions.  The intrinsics
// enter through D' = (i - O_y, j - O_x, F): dL/dF = sum dL/dD'_z,
// dL/dO_x = -sum dL/dD'_y, dL/dO_y = -sum dL/dD'_x.
#include "voge_internal.hpp"
#include "voge_launch.hpp"

namespace voge {

__device__ __forceinline__ double wave_sum_d(double x) {
    for (int off = WAVE / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// One thread per kernel of an item, in original order (the accumulators
// are kept in that order); a block belongs to one item.
__global__ __launch_bounds__(EPI_THREADS) void k_epilogue(BatchDev B) {
    __shared__ double s_red[EPI_THREADS / WAVE][12];
    const int item = B.n_items == 1 ? 0 : B.epi_item[blockIdx.x];
    const ItemDev it = B.items[item];     // a copy, read before any store
    const TraceArgs& A = it.t;
    const int lb = blockIdx.x - it.epi_start;
    const int r = lb * EPI_THREADS + threadIdx.x;       // the kernel's original index
    const bool want_cam = it.grad_camera != nullptr;
    double part[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) part[e] = 0.0;
    if (r < A.N) {
        const size_t n = r;
        double gm[3] = {0.0, 0.0, 0.0};
        double gc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        double M0[3], Sig[6], S0[6];
        bool ok = true;
        for (int d = 0; d < 3; ++d) {
            M0[d] = (double)gp(it.means)[n * 3 + d];
            ok = ok && isfinite(M0[d]);
        }
        for (int e = 0; e < 6; ++e) {
            Sig[e] = (double)gp(it.covs)[n * 6 + e];
            ok = ok && isfinite(Sig[e]);
        }
        ok = ok && spd_inverse6(Sig, S0);
        if (ok) {
            double R[9];
            for (int e = 0; e < 9; ++e) R[e] = (double)it.cam.R[e];
            const auto gM = gp(A.gM) + n * 3;
            const double g0 = gM[0], g1 = gM[1], g2 = gM[2];
            double G[9];
            {
                const auto q = gp(A.gS) + n * 6;
                G[0] = q[0]; G[1] = q[1]; G[2] = q[2];
                G[3] = q[1]; G[4] = q[3]; G[5] = q[4];
                G[6] = q[2]; G[7] = q[4]; G[8] = q[5];
            }
            for (int c = 0; c < 3; ++c) gm[c] = R[c] * g0 + R[3 + c] * g1 + R[6 + c] * g2;   // R^T g
            // X = R^T G R
            double GR[9], X[9];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    GR[3 * a + b] = G[3 * a] * R[b] + G[3 * a + 1] * R[3 + b] + G[3 * a + 2] * R[6 + b];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    X[3 * a + b] = R[a] * GR[b] + R[3 + a] * GR[3 + b] + R[6 + a] * GR[6 + b];
            const double S[9] = {S0[0], S0[1], S0[2], S0[1], S0[3], S0[4], S0[2], S0[4], S0[5]};
            double SX[9], Y[9];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    SX[3 * a + b] = S[3 * a] * X[b] + S[3 * a + 1] * X[3 + b] + S[3 * a + 2] * X[6 + b];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    Y[3 * a + b] = -(SX[3 * a] * S[b] + SX[3 * a + 1] * S[3 + b] + SX[3 * a + 2] * S[6 + b]);
            gc[0] = Y[0];
            gc[1] = Y[1] + Y[3];
            gc[2] = Y[2] + Y[6];
            gc[3] = Y[4];
            gc[4] = Y[5] + Y[7];
            gc[5] = Y[8];
            if (want_cam) {
                // dL/dR = g M0^T + 2 G R S0
                double RS[9];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        RS[3 * a + b] = R[3 * a] * S[b] + R[3 * a + 1] * S[3 + b] + R[3 * a + 2] * S[6 + b];
                const double gv[3] = {g0, g1, g2};
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        part[3 * a + b] = gv[a] * M0[b] +
                                          2.0 * (G[3 * a] * RS[b] + G[3 * a + 1] * RS[3 + b] + G[3 * a + 2] * RS[6 + b]);
                part[9] = g0;
                part[10] = g1;
                part[11] = g2;
            }
        }
        for (int d = 0; d < 3; ++d) gp(it.grad_means)[n * 3 + d] = (float)gm[d];
        for (int e = 0; e < 6; ++e) gp(it.grad_covs)[n * 6 + e] = (float)gc[e];
        const int C = A.C;
        const auto ga = gp(A.gA) + n * C;
        const auto go = gp(it.grad_attrs) + n * C;
        for (int c = 0; c < C; ++c) go[c] = ga[c];
    }
    if (want_cam) {
        const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            const double s = wave_sum_d(part[e]);
            if (lane == 0) s_red[wave][e] = s;
        }
        __syncthreads();
        if (threadIdx.x < 12) {
            double s = 0.0;
            for (int w = 0; w < EPI_THREADS / WAVE; ++w) s += s_red[w][threadIdx.x];
            gp(it.camP)[(size_t)lb * 12 + threadIdx.x] = s;
        }
    }
}

// One block per item, one wave per camera value: a fixed-order reduction of
// the item's per-block and per-tile partials (lane-strided sums, then a
// shuffle tree).
constexpr int FIN_THREADS = 16 * WAVE;

__global__ __launch_bounds__(FIN_THREADS) void k_cam_finalize(BatchDev B) {
    const ItemDev& it = B.items[blockIdx.x];
    if (it.grad_camera == nullptr) return;
    const int e = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    if (e >= 15) return;
    double s = 0.0;
    if (e < 12) {
        for (int b = lane; b < it.n_epi; b += WAVE) s += it.camP[(size_t)b * 12 + e];
    } else {
        const int comp = (e == 12) ? 2 : (e == 13 ? 1 : 0);   // F <- z, O_x <- y, O_y <- x
        for (int t = lane; t < it.t.n_tiles; t += WAVE) s += it.t.tileD[(size_t)t * 3 + comp];
    }
    s = wave_sum_d(s);
    if (lane == 0) it.grad_camera[e] = (float)(e == 13 || e == 14 ? -s : s);
}

// Sampler epilogue (Sec. 3.4, Eq. 10): one thread per kernel divides the
// reduced sum_p W phi by sum_p W (both in original kernel order); a kernel
// that no pixel keeps gets alpha = 0 and weight 0.
__global__ __launch_bounds__(EPI_THREADS) void k_sample_epilogue(BatchDev B) {
    const int item = B.n_items == 1 ? 0 : B.epi_item[blockIdx.x];
    const ItemDev it = B.items[item];     // a copy, read before any store
    const TraceArgs& A = it.t;
    const int r = (blockIdx.x - it.epi_start) * EPI_THREADS + threadIdx.x;
    if (r >= A.N) return;
    const size_t n = r;
    const int C = A.C;
    const float den = gp(A.gW)[n];
    const auto num = gp(A.gA) + n * C;
    const auto out = gp(it.sampled) + n * C;
    if (den > 0.f) {
        for (int c = 0; c < C; ++c) out[c] = num[c] / den;
    } else {
        for (int c = 0; c < C; ++c) out[c] = 0.f;
    }
    if (it.sample_weight) gp(it.sample_weight)[n] = den;
}

hipError_t launch_sample_epilogue(const BatchDev& b, int total_epi, hipStream_t s) {
    if (total_epi > 0) hipLaunchKernelGGL(k_sample_epilogue, dim3(total_epi), dim3(EPI_THREADS), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_epilogue(const BatchDev& b, int total_epi, hipStream_t s) {
    if (total_epi > 0) hipLaunchKernelGGL(k_epilogue, dim3(total_epi), dim3(EPI_THREADS), 0, s, b);
    if (b.n_items > 0) hipLaunchKernelGGL(k_cam_finalize, dim3(b.n_items), dim3(FIN_THREADS), 0, s, b);
    return hipGetLastError();
}

}  // namespace voge
