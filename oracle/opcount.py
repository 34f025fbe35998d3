"""Algorithmic operation counts of a workload, from the FP64 oracle.

TEST INFRASTRUCTURE: runs only the oracle.  Renders every pixel of the
workload with the oracle and records, over the whole image, the number of
rays, of (ray, passing kernel) pairs, and sum K_eff and sum K_eff^2 of the kept
sets -- the units the per-step FLOP constants of ``oracle.py`` multiply.
The result is written next to this file as ``opcount_<workload>.json``.

    python -m oracle.opcount            # the 512x512 torus workload
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


def count(job) -> dict:
    cam = job.camera
    t0 = time.time()
    r = O.forward(job.scene.means, job.scene.covs, job.scene.attrs, cam.as_vector(), cam.height, cam.width,
                  job.K, job.eta)
    ke = r.k_eff.astype(np.int64)
    C = job.scene.channels
    out = {
        "workload": job.name,
        "rays": int(cam.height * cam.width),
        "sum_n_pass": int(r.n_pass.astype(np.int64).sum()),
        "sum_k_eff": int(ke.sum()),
        "sum_k_eff_sq": int((ke * ke).sum()),
        "hit_rays": int((ke > 0).sum()),
        "channels": C,
        "flop_trace_per_pass": O.FLOP_TRACE,
        "flop_pair": O.FLOP_PAIR,
        "flop_kept": O.flop_kept(C),
        "flop_bpair": O.FLOP_BPAIR,
        "flop_bkept": O.flop_bkept(C),
    }
    out["flop_select"] = O.FLOP_TRACE * out["sum_n_pass"]
    out["flop_blend"] = O.FLOP_PAIR * out["sum_k_eff_sq"] + O.flop_kept(C) * out["sum_k_eff"]
    out["flop_bwd"] = O.backward_flops(ke, C)
    out["flop_bwd_pixel"] = O.FLOP_BPAIR * out["sum_k_eff_sq"] + O.flop_bkept_pixel(C) * out["sum_k_eff"]
    out["flop_bwd_chain"] = O.flop_bkept_chain(C) * out["sum_k_eff"]
    out["flop_forward"] = O.forward_flops(r.n_pass, ke, C)
    out["flop_per_ray_fwd_bwd"] = (out["flop_forward"] + out["flop_bwd"]) / out["rays"]
    out["oracle_seconds"] = round(time.time() - t0, 2)
    return out


def path_for(name: str) -> str:
    return os.path.join(HERE, f"opcount_{name}.json")


def main():
    job = S.config_torus()
    res = count(job)
    with open(path_for(job.name), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
