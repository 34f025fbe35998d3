"""Comparison rules between the GPU library and the FP64 oracle.

Tolerance (the hot path's stated bar: 1e-5 relative in FP32; kept sets exact
except for near ties):
  * images: |C_gpu - C_ref| <= RTOL * (|C_ref| + sum_k W_k |c_k|) per element,
    the floor being the oracle's absolute blend sum (C can cancel);
  * kept sets: equal, except at pixels the oracle flags (a near tie at the
    K-th place within 1e-6 relative in l, or a kernel within 1e-5 of the
    threshold ln eta); such pixels are left out of the element comparison;
  * gradients: |g - g_ref| <= RTOL * (sum over pixels of |contribution|)
    per element, and ||g - g_ref||_inf <= RTOL ||g_ref||_inf per tensor --
    except that the tensor-wide bound is never below FP32's resolution on
    the largest absolute sum, F32_FLOOR * ||abs sum||_inf: where a gradient
    element is a sum whose terms cancel (kernels a few thousandths wide seen
    by many pixels), no FP32 arithmetic gets within 1e-5 of the small result.
"""

import numpy as np
import torch

RTOL = 1e-5
F32_FLOOR = 1e-7     # a little above FP32's unit roundoff (6e-8)


def to_dev(a, device="cuda"):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).to(device)


def compare_images(img_gpu, ref_image, ref_absum, rtol=RTOL, mask=None):
    """img_gpu, ref_image, ref_absum: (n, C).  Returns max ratio err/bound."""
    g = np.asarray(img_gpu, np.float64)
    r = np.asarray(ref_image, np.float64)
    bound = rtol * (np.abs(r) + np.asarray(ref_absum, np.float64)) + 1e-30
    err = np.abs(g - r)
    if mask is not None:
        err = err[mask]
        bound = bound[mask]
    ratio = (err / bound).max() if err.size else 0.0
    return float(ratio)


def compare_kept(kept_gpu, ref_kept, ref_flags, ref_l=None):
    """Kept sets as sets: both (n, K) int arrays, -1 padded.  The order inside
    a set is not part of the result (the blend is order-free); when ref_l
    (n, K) is given, the GPU order must still be ascending in the oracle's l,
    up to ties within 1e-6 relative.
    Returns (n mismatching pixels, n mismatching unflagged pixels, mask of equal)."""
    kg = np.sort(np.asarray(kept_gpu), axis=1)
    kr = np.sort(np.asarray(ref_kept), axis=1)
    same = np.all(kg == kr, axis=1)
    bad_unflagged = (~same) & (np.asarray(ref_flags) == 0)
    if ref_l is not None:
        kgo = np.asarray(kept_gpu)
        kro = np.asarray(ref_kept)
        for p in np.flatnonzero(same):
            lut = {int(i): float(l) for i, l in zip(kro[p], ref_l[p]) if i >= 0}
            ls = [lut[int(i)] for i in kgo[p] if i >= 0]
            for a, b in zip(ls, ls[1:]):
                assert b >= a - 1e-6 * abs(a), ("kept list not ascending in l", p, ls)
    return int((~same).sum()), int(bad_unflagged.sum()), same


def compare_grad(g, ref, ref_abs, rtol=RTOL):
    """Returns (max per-element ratio, inf-norm ratio)."""
    g = np.asarray(g, np.float64).reshape(-1)
    r = np.asarray(ref, np.float64).reshape(-1)
    a = np.asarray(ref_abs, np.float64).reshape(-1)
    err = np.abs(g - r)
    bound = rtol * a + 1e-30
    elem = float((err / bound).max()) if err.size else 0.0
    inf_bound = max(rtol * np.abs(r).max(), F32_FLOOR * a.max()) + 1e-30 if err.size else 1.0
    inf = float(err.max() / inf_bound) if err.size else 0.0
    return elem, inf
