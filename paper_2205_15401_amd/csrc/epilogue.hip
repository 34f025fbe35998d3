// epilogue.hip -- backward epilogue (FP64): camera-space gradients of each
// kernel back to world space, and the camera gradient.
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

__global__ __launch_bounds__(EPI_THREADS) void k_epilogue(EpiArgs A) {
    __shared__ double s_red[EPI_THREADS / WAVE][12];
    const int r = blockIdx.x * EPI_THREADS + threadIdx.x;
    double part[12];
#pragma unroll
    for (int e = 0; e < 12; ++e) part[e] = 0.0;
    if (r < A.N) {
        const size_t n = A.rec[r].idx;
        double gm[3] = {0.0, 0.0, 0.0};
        double gc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        double M0[3], Sig[6], S0[6];
        bool ok = true;
        for (int d = 0; d < 3; ++d) {
            M0[d] = (double)A.means[n * 3 + d];
            ok = ok && isfinite(M0[d]);
        }
        for (int e = 0; e < 6; ++e) {
            Sig[e] = (double)A.covs[n * 6 + e];
            ok = ok && isfinite(Sig[e]);
        }
        ok = ok && spd_inverse6(Sig, S0);
        if (ok) {
            double R[9];
            for (int e = 0; e < 9; ++e) R[e] = (double)A.cam.R[e];
            const double g0 = A.gM[(size_t)r * 3], g1 = A.gM[(size_t)r * 3 + 1], g2 = A.gM[(size_t)r * 3 + 2];
            const double* gs = nullptr;
            (void)gs;
            double G[9];
            {
                const float* q = A.gS + (size_t)r * 6;
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
            if (A.grad_camera) {
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
        for (int d = 0; d < 3; ++d) A.grad_means[n * 3 + d] = (float)gm[d];
        for (int e = 0; e < 6; ++e) A.grad_covs[n * 6 + e] = (float)gc[e];
    }
    if (A.grad_camera) {
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
            A.camP[(size_t)blockIdx.x * 12 + threadIdx.x] = s;
        }
    }
}

// One wave per camera value: a fixed-order reduction of the per-block and
// per-tile partials (lane-strided sums, then a shuffle tree).
constexpr int FIN_THREADS = 16 * WAVE;

__global__ __launch_bounds__(FIN_THREADS) void k_cam_finalize(EpiArgs A, int nblk) {
    const int e = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    if (e >= 15) return;
    double s = 0.0;
    if (e < 12) {
        for (int b = lane; b < nblk; b += WAVE) s += A.camP[(size_t)b * 12 + e];
    } else {
        const int comp = (e == 12) ? 2 : (e == 13 ? 1 : 0);   // F <- z, O_x <- y, O_y <- x
        for (int t = lane; t < A.n_tiles; t += WAVE) s += A.tileD[(size_t)t * 3 + comp];
    }
    s = wave_sum_d(s);
    if (lane == 0) A.grad_camera[e] = (float)(e == 13 || e == 14 ? -s : s);
}

hipError_t launch_epilogue(const EpiArgs& a, hipStream_t s) {
    const int nblk = (a.N + EPI_THREADS - 1) / EPI_THREADS;
    if (nblk > 0) hipLaunchKernelGGL(k_epilogue, dim3(nblk), dim3(EPI_THREADS), 0, s, a);
    if (a.grad_camera) hipLaunchKernelGGL(k_cam_finalize, dim3(1), dim3(FIN_THREADS), 0, s, a, nblk);
    return hipGetLastError();
}

}  // namespace voge
