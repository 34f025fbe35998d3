"""Algorithmic operation counts of a workload, from the FP64 oracle.

TEST INFRASTRUCTURE: runs only the oracle.  Renders every pixel of the
workload with the oracle and records, over the whole image, the number of
rays, of (ray, passing kernel) pairs, and sum K_eff and sum K_eff^2 of the kept
sets -- the units the per-step FLOP constants of ``oracle.py`` multiply.
The result is written next to this file as ``opcount_<workload>.json``.

    python -m oracle.opcount            # the 512x512 torus workload
    python -m oracle.opcount poses      # 256 poses of the 4,096-kernel torus at 128x128
"""

from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import oracle as O  # noqa: E402
from paper_2205_15401_amd import scenes as S  # noqa: E402


def count(jobs, name: str) -> dict:
    """Counts over every ray of every job (all jobs share C)."""
    if not isinstance(jobs, (list, tuple)):
        jobs = [jobs]
    t0 = time.time()
    kes, n_pass, rays = [], 0, 0
    for job in jobs:
        cam = job.camera
        r = O.forward(job.scene.means, job.scene.covs, job.scene.attrs, cam.as_vector(), cam.height, cam.width,
                      job.K, job.eta)
        kes.append(r.k_eff.astype(np.int64))
        n_pass += int(r.n_pass.astype(np.int64).sum())
        rays += cam.height * cam.width
    ke = np.concatenate(kes)
    C = jobs[0].scene.channels
    out = {
        "workload": name,
        "renders": len(jobs),
        "rays": int(rays),
        "sum_n_pass": n_pass,
        "sum_k_eff": int(ke.sum()),
        "sum_k_eff_sq": int((ke * ke).sum()),
        "hit_rays": int((ke > 0).sum()),
        "channels": C,
        "flop_trace_per_pass": O.FLOP_TRACE,
        "flop_pair": O.FLOP_PAIR,
        "flop_kept": O.flop_kept(C),
        "flop_bpair": O.FLOP_BPAIR,
        "flop_bkept": O.flop_bkept(C),
        "flop_quad_pair": O.FLOP_QUAD_PAIR,
        "flop_quad_sample": O.FLOP_QUAD_SAMPLE,
    }
    out["flop_select"] = O.FLOP_TRACE * out["sum_n_pass"]
    out["flop_blend"] = O.FLOP_PAIR * out["sum_k_eff_sq"] + O.flop_kept(C) * out["sum_k_eff"]
    out["flop_bwd"] = O.backward_flops(ke, C)
    out["flop_bwd_pixel"] = O.FLOP_BPAIR * out["sum_k_eff_sq"] + O.flop_bkept_pixel(C) * out["sum_k_eff"]
    out["flop_bwd_chain"] = O.flop_bkept_chain(C) * out["sum_k_eff"]
    # the sampler: the forward's blend without the colour sum, then the pair reduction
    out["flop_blend_weights"] = out["flop_blend"] - 2 * C * out["sum_k_eff"]
    out["flop_sample_reduce"] = O.flop_sample(C) * out["sum_k_eff"]
    out["flop_forward"] = O.FLOP_TRACE * n_pass + out["flop_blend"]
    out["flop_per_ray_fwd_bwd"] = (out["flop_forward"] + out["flop_bwd"]) / out["rays"]
    out["oracle_seconds"] = round(time.time() - t0, 2)
    return out


def path_for(name: str) -> str:
    return os.path.join(HERE, f"opcount_{name}.json")


POSES_NAME = "torus4096_256poses_128px_C3_K20"


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "poses":
        res = count(S.config_poses(), POSES_NAME)
    else:
        job = S.config_torus()
        res = count(job, job.name)
    with open(path_for(res["workload"]), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
