"""Comparison rules between the GPU library and the FP64 oracle.

Tolerance (the hot path's stated bar: 1e-5 relative in FP32; kept sets exact
except for near ties):
  * kept sets: equal as sets, except at pixels the oracle flags (a near tie
    at the K-th place within 1e-6 relative in l, or a kernel within 1e-5 of
    the threshold ln eta); there every kernel in which the two sets differ
    must itself be such a near tie or near-threshold kernel;
  * images: every pixel, flagged or not, against the oracle's blend (Eq. 7-8)
    of the GPU's own kept set (at unflagged pixels that set is the oracle's):
    |C_gpu - C_ref| <= RTOL * (|C_ref| + sum_k W_k |c_k|) per element, the
    floor being the oracle's absolute blend sum (C can cancel);
  * gradients: against the oracle's backward on the GPU's kept sets, every
    pixel included: |g - g_ref| <= RTOL * (sum over pixels of |contribution|)
    per element, and per tensor ||g - g_ref||_inf <= max(RTOL ||g_ref||_inf,
    FLOOR_MULT x the FP32 noise floor), the floor measured in the same check:
    the largest spread of the oracle's backward over a few draws in which
    every FP32 input moves by one ulp (check_backward_vs_oracle).  Where
    that floor exceeds RTOL (cancelling tensors: the covariance gradients of
    thin, rotated kernels, whose sums of absolute contributions are hundreds
    of times the gradient's largest value) no FP32 code meets the RTOL
    tensor-wide bar; the check then holds the GPU to FLOOR_MULT = 8 measured
    spreads.  An FP32 implementation's error in such an element is a few
    units of roundoff of its absolute contribution sum (the per-element rule
    bounds it; the GPU sits at ~2e-7 of it), while one input-ulp draw moves
    it by one such unit or less, and a maximum over one or two draws is a low
    estimate; measured GPU errors are 1.4-4.7 two-draw floors on the cloud
    scenes.  The per-element rule is unchanged and binding.  The plain
    ||g - g_ref||_inf / ||g_ref||_inf of every check is recorded beside the
    floor (VOGE_PARITY_LOG).

The measured floor (tests/golden/fp32_noise_floor.json, written by
oracle/noise_floor.py from the oracle alone): one-ulp moves of the scene
geometry or the camera change the oracle's images by up to 1.2e-4 of the
image scale and its gradients by up to 1.2e-4 (centres), 2.1e-4
(covariances), 4.6e-5 (attributes) and 9e-5 (camera) of ||g||_inf on the
512^2 torus, the 256-pose torus and the uneven clouds -- the 1e-5 bar lies
below it; one-ulp moves of attributes and upstream gradient alone change
them by ~1e-7.  The GPU path meets the image rule at every pixel because it
traces in FP64 from the exact FP32 inputs.

GPU-vs-GPU gradient comparisons (compare_grad) keep the tensor-wide floor
F32_FLOOR * ||abs sum||_inf: a little above FP32's unit roundoff on the
largest absolute sum, which is below the measured spread of every tensor
but the covariances'.
"""

import json
import math
import os

import numpy as np
import torch

RTOL = 1e-5
F32_FLOOR = 1e-7     # a little above FP32's unit roundoff (6e-8)
FLOOR_MULT = 8.0     # tensor-wide gradient bound: this many measured one-ulp spreads
NEAR_TIE = 1e-6      # relative l difference of a near tie at the K-th place
NEAR_ETA = 1e-5      # |q - ln eta| of a near-threshold kernel

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def to_dev(a, device="cuda"):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).to(device)


def record(test, **values):
    """Append measured errors to the file named by VOGE_PARITY_LOG (JSON lines)."""
    path = os.environ.get("VOGE_PARITY_LOG")
    if not path:
        return
    with open(path, "a") as f:
        f.write(json.dumps({"test": test, **values}) + "\n")


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
                assert b >= a - NEAR_TIE * abs(a), ("kept list not ascending in l", p, ls)
    return int((~same).sum()), int(bad_unflagged.sum()), same


def explain_set_differences(own, given, eta, K, rows):
    """At pixels `rows`, where the GPU's kept set differs from the oracle's
    own selection, check that each kernel in which they differ is one the
    parity rule lets go either way: within NEAR_ETA of the threshold, or a
    near tie at the K-th place (within NEAR_TIE relative of the other set's
    K-th depth when that set is full).  own: the oracle's forward with its
    own selection; given: the oracle's forward on the GPU's sets (the same
    pixel order).  Returns the number of kernels so explained."""
    ln_eta = math.log(eta)
    n = 0
    for p in rows:
        o_idx, g_idx = own.kept_idx[p], given.kept_idx[p]
        o = {int(i): own.kept_rec[p, s] for s, i in enumerate(o_idx) if i >= 0}
        g = {int(i): given.kept_rec[p, s] for s, i in enumerate(g_idx) if i >= 0}
        o_kth = max(r[0] for r in o.values()) if len(o) == K else math.inf
        g_kth = max(r[0] for r in g.values()) if len(g) == K else math.inf
        for i, r in g.items():
            l, q = float(r[0]), float(r[1])
            assert l > 0 and q > ln_eta - NEAR_ETA, ("GPU kept a kernel that does not pass", p, i, l, q)
        for i in set(g) - set(o):
            l, q = float(g[i][0]), float(g[i][1])
            ok = abs(q - ln_eta) <= NEAR_ETA or l <= o_kth * (1 + NEAR_TIE)
            assert ok, ("GPU keeps a kernel the oracle does not, and it is no near tie", p, i, l, q, o_kth)
            n += 1
        for i in set(o) - set(g):
            l, q = float(o[i][0]), float(o[i][1])
            ok = abs(q - ln_eta) <= NEAR_ETA or l >= g_kth * (1 - NEAR_TIE)
            assert ok, ("GPU drops a kernel the oracle keeps, and it is no near tie", p, i, l, q, g_kth)
            n += 1
    return n


def grad_errors(g, ref, ref_abs, rtol=RTOL):
    """(max per-element ratio, inf-norm ratio, plain ||g - ref||_inf / ||ref||_inf)."""
    g = np.asarray(g, np.float64).reshape(-1)
    r = np.asarray(ref, np.float64).reshape(-1)
    a = np.asarray(ref_abs, np.float64).reshape(-1)
    if not g.size:
        return 0.0, 0.0, 0.0
    err = np.abs(g - r)
    bound = rtol * a + 1e-30
    elem = float((err / bound).max())
    inf_bound = max(rtol * np.abs(r).max(), F32_FLOOR * a.max()) + 1e-30
    inf = float(err.max() / inf_bound)
    plain = float(err.max() / (np.abs(r).max() + 1e-300))
    return elem, inf, plain


def compare_grad(g, ref, ref_abs, rtol=RTOL):
    """Returns (max per-element ratio, inf-norm ratio)."""
    elem, inf, _ = grad_errors(g, ref, ref_abs, rtol)
    return elem, inf


# --------------------------------------------------------------------------
# whole checks: GPU outputs against the oracle on the GPU's own kept sets


def _oracle():
    from oracle import oracle as O
    return O


def check_forward_vs_oracle(img, wsum, kept, scene, cam, K, eta=0.01, pixels=None, max_flagged_frac=0.01,
                            name="", order=True, full_image=False):
    """img (H*W, C) or None, wsum (H*W,) or None, kept (H*W, K): the GPU's
    forward outputs.  Checks, at `pixels` (None: every pixel), the kept sets
    against the oracle's own selection (differences only where flagged, and
    each explained) and the image and weight sum at every checked pixel
    against the oracle's blend of the GPU's kept set; with full_image, the
    image and weight sum of every pixel of the image as well (the blend of a
    given set costs K^2 per pixel, not N).  Returns (own, given) oracle
    results, given in the order of `pixels`."""
    O = _oracle()
    cv = cam.as_vector()
    H, W = cam.height, cam.width
    sel = np.arange(H * W) if pixels is None else np.asarray(pixels)
    own = O.forward(scene.means, scene.covs, scene.attrs, cv, H, W, K, eta, pixels=pixels)
    kg = np.ascontiguousarray(np.asarray(kept).reshape(H * W, K)[sel])
    n_bad, n_bad_unflagged, same = compare_kept(kg, own.kept_idx, own.flags,
                                                own.kept_rec[..., 0] if order else None)
    assert n_bad_unflagged == 0, f"{name}: {n_bad_unflagged} unflagged pixels with different kept sets"
    assert n_bad <= max_flagged_frac * len(sel) + 1, f"{name}: {n_bad} flagged pixels differ"
    given = O.forward(scene.means, scene.covs, scene.attrs, cv, H, W, K, eta, pixels=pixels, given=kg)
    n_expl = explain_set_differences(own, given, eta, K, np.flatnonzero(~same))
    rep = {"pixels": int(len(sel)), "flagged": int((own.flags != 0).sum()), "sets_differ": n_bad,
           "kernels_explained": n_expl}
    if img is not None:
        ig = np.asarray(img, np.float64).reshape(H * W, -1)[sel]
        r_img = compare_images(ig, given.image, given.absum)
        scale = np.abs(given.image).max() + 1e-300
        rep.update(image_ratio=r_img, image_plain=float(np.abs(ig - given.image).max() / scale))
        assert r_img <= 1.0, f"{name}: image error {r_img:.3g} x tolerance"
    if wsum is not None:
        wg = np.asarray(wsum, np.float64).reshape(-1)[sel, None]
        r_ws = compare_images(wg, given.wsum[:, None], given.wsum[:, None])
        rep.update(wsum_ratio=r_ws)
        assert r_ws <= 1.0, f"{name}: weight-sum error {r_ws:.3g} x tolerance"
    if full_image and pixels is not None:
        kall = np.ascontiguousarray(np.asarray(kept).reshape(H * W, K))
        ga = O.forward(scene.means, scene.covs, scene.attrs, cv, H, W, K, eta, given=kall)
        if img is not None:
            r_all = compare_images(np.asarray(img, np.float64).reshape(H * W, -1), ga.image, ga.absum)
            rep.update(image_ratio_all_pixels=r_all)
            assert r_all <= 1.0, f"{name}: image error {r_all:.3g} x tolerance (all pixels)"
        if wsum is not None:
            r_all = compare_images(np.asarray(wsum, np.float64).reshape(-1, 1), ga.wsum[:, None], ga.wsum[:, None])
            assert r_all <= 1.0, f"{name}: weight-sum error {r_all:.3g} x tolerance (all pixels)"
    record(name or "forward", **rep)
    return own, given


def ulp_jitter(a, rng):
    """Each FP32 element moved one ulp up or down at random (zeros stay)."""
    a = np.asarray(a, np.float32)
    up = rng.random(a.shape) < 0.5
    out = np.where(up, np.nextafter(a, np.float32(np.inf)), np.nextafter(a, np.float32(-np.inf)))
    return np.where(a == 0, a, out).astype(np.float32)


GRAD_NAMES = ("means", "covs", "attrs", "camera")


def check_backward_vs_oracle(grads, scene, cam, K, G, kept, eta=0.01, pixels=None, mode=0, name="",
                             floor_draws=2, seed=0):
    """grads: dict name -> GPU gradient array (any of means, covs, attrs,
    camera).  G: the upstream gradient at `pixels` ((n, C); pixels None: the
    whole image), kept: the GPU's kept sets (H*W, K).  The oracle's backward
    on the GPU's kept sets is the reference for every element.  Per tensor the
    inf-norm bound is max(RTOL ||g_ref||_inf, FLOOR_MULT x the FP32 noise
    floor), the floor being measured here: the spread of the same oracle backward when
    every FP32 input (scene, camera, upstream gradient) moves by one ulp
    (floor_draws draws).  Returns {name: (elem ratio, inf ratio, plain rel)}."""
    O = _oracle()
    cv = cam.as_vector()
    H, W = cam.height, cam.width
    sel = np.arange(H * W) if pixels is None else np.asarray(pixels)
    kg = np.ascontiguousarray(np.asarray(kept).reshape(H * W, K)[sel])
    C = scene.attrs.shape[1]
    Gs = np.asarray(G, np.float32).reshape(len(sel), C)
    ref = O.backward(scene.means, scene.covs, scene.attrs, cv, H, W, K, Gs, eta, pixels=pixels, mode=mode,
                     given=kg)
    rng = np.random.default_rng(seed + 9001)
    floor = {n: 0.0 for n in GRAD_NAMES}
    for _ in range(floor_draws):
        b = O.backward(ulp_jitter(scene.means, rng), ulp_jitter(scene.covs, rng), ulp_jitter(scene.attrs, rng),
                       ulp_jitter(cv, rng), H, W, K, ulp_jitter(Gs, rng), eta, pixels=pixels, mode=mode, given=kg)
        for n in GRAD_NAMES:
            floor[n] = max(floor[n], float(np.abs(getattr(b, n) - getattr(ref, n)).max(initial=0.0)))
    out = {}
    rep = {}
    for n, g in grads.items():
        r, a = getattr(ref, n), getattr(ref, "abs_" + n)
        gg = np.asarray(g, np.float64).reshape(-1)
        rr = np.asarray(r, np.float64).reshape(-1)
        err = np.abs(gg - rr)
        elem = float((err / (RTOL * np.asarray(a).reshape(-1) + 1e-30)).max(initial=0.0))
        inf_bound = max(RTOL * np.abs(rr).max(initial=0.0), FLOOR_MULT * floor[n]) + 1e-30
        inf = float(err.max(initial=0.0) / inf_bound)
        plain = float(err.max(initial=0.0) / (np.abs(rr).max(initial=0.0) + 1e-300))
        floor_rel = floor[n] / (np.abs(rr).max(initial=0.0) + 1e-300)
        out[n] = (elem, inf, plain)
        rep[n] = {"elem_ratio": elem, "inf_ratio": inf, "plain_rel": plain, "floor_rel": floor_rel}
        assert elem <= 1.0 and inf <= 1.0, (f"{name} {n}: element {elem:.3g}, inf-norm {inf:.3g} x tolerance "
                                            f"(plain {plain:.3g}, floor {floor_rel:.3g})")
    record(name or "backward", **rep)
    return out
