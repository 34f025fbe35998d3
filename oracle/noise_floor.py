"""The FP32 noise floor of the rendering equations, measured with the oracle.

TEST INFRASTRUCTURE ONLY (calls the FP64 oracle and the seeded scene
generators, nothing else).

Every input of the GPU path is an FP32 number, and every FP32 computation of
the method rounds what it derives from those inputs at the level of one unit
in the last place.  Running the FP64 oracle on inputs moved by one ulp (each
element independently up or down) and comparing with the unmoved inputs shows
how far the exact result moves under such a rounding: no FP32 implementation
can be held closer to the oracle than that.  Kept sets are held fixed (the
unmoved selection is handed to the perturbed runs), so the spread is that of
the blend (Eq. 7-8) and of its gradients, not of the discrete selection.

An FP32 implementation also rounds what it derives per (pixel, kernel) pair:
the oracle's jitter mode moves each per-pair derivative of the backward
(dL/dq, dL/dl, dL/da and the pair's weight in the attribute gradient) by one
FP32 unit roundoff, up or down, which no implementation that carries them in
FP32 avoids.

For each workload and each group of quantities moved (all inputs; the scene
geometry; the camera; attributes and upstream gradient; the per-pair
derivatives alone; all inputs and the per-pair derivatives) this writes, per
output, the largest spread over a few perturbation draws in the units the
parity rules use:
  * image: max |dC| / (|C| + sum_k W_k |c_k|)   (the per-element image scale);
  * each gradient tensor: max |dg| / ||g||_inf, max |dg| / ||abs||_inf and the
    per-element max |dg| / abs (abs: the oracle's absolute-contribution sums).

Usage: python -m oracle.noise_floor [--quick]  ->  tests/golden/fp32_noise_floor.json
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2205_15401_amd import scenes as S  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "fp32_noise_floor.json")


def ulp_jitter(a: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """Each FP32 element moved one ulp up or down at random (zeros stay)."""
    a = np.asarray(a, np.float32)
    up = rng.random(a.shape) < 0.5
    out = np.where(up, np.nextafter(a, np.float32(np.inf)), np.nextafter(a, np.float32(-np.inf)))
    return np.where(a == 0, a, out).astype(np.float32)


GROUPS = {
    "all": ("means", "covs", "attrs", "camera", "grad"),
    "geometry": ("means", "covs"),
    "camera": ("camera",),
    "attrs_grad": ("attrs", "grad"),
    # the per-pair derivatives of the backward rounded to FP32 (the oracle's
    # jitter mode), alone and on top of every input
    "pairs": ("pairs",),
    "all_with_pairs": ("means", "covs", "attrs", "camera", "grad", "pairs"),
}


def spread(scene, cam, K, pixels, G, draws, rng, eta=0.01, group="all"):
    """Max spread of image and gradients over `draws` one-ulp perturbations of
    the inputs in `group` (scene geometry, attributes, camera, upstream
    gradient) with the kept sets fixed."""
    moved = GROUPS[group]
    cv = cam.as_vector()
    H, W = cam.height, cam.width
    base = O.forward(scene.means, scene.covs, scene.attrs, cv, H, W, K, eta, pixels=pixels)
    given = base.kept_idx
    bb = O.backward(scene.means, scene.covs, scene.attrs, cv, H, W, K, G, eta, pixels=pixels, given=given)
    img_scale = np.abs(base.image) + base.absum
    res = {"image_rel": 0.0}
    names = ("means", "covs", "attrs", "camera")
    for n in names:
        res[n] = {"inf_over_ref": 0.0, "inf_over_abs": 0.0, "elem_over_abs": 0.0}
    for _ in range(draws):
        jit = lambda x, name: ulp_jitter(x, rng) if name in moved else np.asarray(x, np.float32)  # noqa: E731
        m, c, a = jit(scene.means, "means"), jit(scene.covs, "covs"), jit(scene.attrs, "attrs")
        cvp = jit(cv, "camera")
        Gp = jit(G, "grad")
        f = O.forward(m, c, a, cvp, H, W, K, eta, pixels=pixels, given=given)
        hit = img_scale > 0
        if hit.any():
            res["image_rel"] = max(res["image_rel"], float((np.abs(f.image - base.image)[hit] / img_scale[hit]).max()))
        seed = int(rng.integers(1, 2**63)) if "pairs" in moved else 0
        b = O.backward(m, c, a, cvp, H, W, K, Gp, eta, pixels=pixels, given=given, jitter_seed=seed)
        for n in names:
            g0, g1 = getattr(bb, n).reshape(-1), getattr(b, n).reshape(-1)
            ab = getattr(bb, "abs_" + n).reshape(-1)
            d = np.abs(g1 - g0)
            r = res[n]
            r["inf_over_ref"] = max(r["inf_over_ref"], float(d.max() / max(np.abs(g0).max(), 1e-300)))
            r["inf_over_abs"] = max(r["inf_over_abs"], float(d.max() / max(ab.max(), 1e-300)))
            nz = ab > 0
            if nz.any():
                r["elem_over_abs"] = max(r["elem_over_abs"], float((d[nz] / ab[nz]).max()))
    res["pixels"] = int(len(pixels))
    res["kept_pairs"] = int((given >= 0).sum())
    return res


def workloads(quick: bool):
    """(name, scene, camera, K, pixel sample) for the three shapes the parity
    rules are stated on: the 512^2 torus, the 256-pose torus, the uneven
    cloud batch."""
    rng = np.random.default_rng(77)
    job = S.config_torus()
    npx = 3000 if quick else 20000
    yield ("torus10000_512px_C16_K20", job.scene, job.camera, job.K,
           rng.choice(512 * 512, npx, replace=False), job.grad_image)
    for job in S.config_poses(n_poses=4 if not quick else 2):
        H = job.camera.height
        yield (f"torus4096_128px_C3_K20_{job.name}", job.scene, job.camera, job.K,
               np.arange(H * H), job.grad_image)
    jobs = S.config_uneven()
    picks = [0, 1, 2, 3] if not quick else [0, 1]
    for s in picks:
        job = jobs[s]
        H = job.camera.height
        n = min(H * H, 4000 if not quick else 1500)
        yield (job.name, job.scene, job.camera, job.K, rng.choice(H * H, n, replace=False), job.grad_image)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="fewer pixels and draws (a check, not the stored numbers)")
    ap.add_argument("--draws", type=int, default=3)
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args(argv)
    rng = np.random.default_rng(2024)
    out = {"what": "spread of the FP64 oracle under one-ulp perturbations of every FP32 input, kept sets fixed",
           "draws": args.draws, "workloads": {}}
    for name, sc, cam, K, pix, G in workloads(args.quick):
        t0 = time.time()
        C = sc.attrs.shape[1]
        Gs = np.asarray(G, np.float32).reshape(-1, C)[pix]
        out["workloads"][name] = {}
        for group in GROUPS:
            r = spread(sc, cam, K, pix, Gs, args.draws, rng, group=group)
            out["workloads"][name][group] = r
            print(f"{name} [{group}]: image {r['image_rel']:.3g}; " + "; ".join(
                f"{n} {r[n]['inf_over_ref']:.3g}/{r[n]['inf_over_abs']:.3g}/{r[n]['elem_over_abs']:.3g}"
                for n in ("means", "covs", "attrs", "camera")) + f"  ({time.time() - t0:.1f} s)", flush=True)
    out["max"] = {}
    for group in GROUPS:
        ws = [w[group] for w in out["workloads"].values()]
        summ = {"image_rel": max(w["image_rel"] for w in ws)}
        for n in ("means", "covs", "attrs", "camera"):
            summ[n] = {k: max(w[n][k] for w in ws) for k in ("inf_over_ref", "inf_over_abs", "elem_over_abs")}
        out["max"][group] = summ
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
