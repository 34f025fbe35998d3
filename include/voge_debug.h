/*
 * voge_debug.h -- diagnostic entry points of libvoge (not needed to render).
 */
#ifndef VOGE_DEBUG_H
#define VOGE_DEBUG_H

#include <stdint.h>

#include "voge.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Accumulated device time of one phase of the library's calls. */
typedef struct voge_phase_time {
    char name[32];            /* "prep", "select", "blend", "zero", "bwd", "fwdbwd", "epilogue" */
    double total_ms;          /* sum of the phase's durations (HIP events)             */
    int64_t count;            /* number of timed calls                                 */
} voge_phase_time_t;

/* Turn per-phase timing on or off for calls made through `ctx`.  When on,
 * every call records a HIP event before and after each phase on the caller's
 * stream: "select" is the single kernel k_select_wave (one wave per 8x8
 * block, launches of 2,048 tiles or more) or k_select (a tile per
 * workgroup; with coarse-stage bins), "blend" k_blend, "bwd" k_bwd,
 * "fwdbwd" k_fwdbwd (the blend and the backward in one kernel, for calls
 * that ask for both); "prep" groups the per-kernel preparation, the depth
 * sort and the block masks, "epilogue" the world-space epilogue.  Host
 * memory only.
 * Returns 0 or VOGE_EINVAL. */
int voge_profile_enable(voge_ctx_t* ctx, int enable);

/* Wait for the recorded events, add their durations to per-phase totals and
 * copy up to max_out totals into `out` (host array); *n_out receives the
 * number of phases seen.  reset != 0 clears the totals afterwards.
 * Synchronises on the recorded events.  Returns 0, VOGE_EINVAL or VOGE_EHIP. */
int voge_profile_read(voge_ctx_t* ctx, voge_phase_time_t* out, int max_out, int* n_out, int reset);

/* Evaluate, on the device, the library's approximation of
 *   Phi(x) = (1 + erf x) / 2,
 * the normal-CDF factor of the erf-sum transmittance (VoGE Eq. 7; App. A.2),
 * for n values.  x and y are device pointers to n floats (y is overwritten).
 * The approximation: erfc(z) = t Q(t) e^{-z^2}, t = 1/(1 + z/2), z = |x|,
 * with Q a degree-8 polynomial fitted to e^{z^2} erfc(z) / t (relative
 * error 4.5e-8; absolute error of Phi in FP32 below 2e-7).
 * Asynchronous on `stream`.  Returns 0, or VOGE_EINVAL (n < 0, or null
 * pointers with n > 0) / VOGE_EHIP. */
int voge_debug_phi(const float* x, float* y, int n, void* stream);

/* The coarse-stage bin choice of calls through `ctx` that do not take a
 * tuned choice (VOGE_TUNED): 0 no bins (the default), 1 bins for scenes of
 * 16,384 kernels or more, 2 bins for every scene.  Results do not depend on it
 * (a tile without a bin scans every kernel of its scene); it selects which
 * code path renders, for tests and timing.  Returns 0 or VOGE_EINVAL. */
int voge_debug_bins(voge_ctx_t* ctx, int bins);

#ifdef __cplusplus
}
#endif

#endif /* VOGE_DEBUG_H */
