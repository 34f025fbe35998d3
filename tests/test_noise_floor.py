"""The FP32 noise floor measurement (oracle/noise_floor.py) on the CPU: its
perturbation moves every element by exactly one ulp, and the stored numbers
(tests/golden/fp32_noise_floor.json) are reproduced by a fresh, smaller run."""

import json
import os

import numpy as np

from oracle import noise_floor as NF
from paper_2205_15401_amd import scenes as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fp32_noise_floor.json")


def test_ulp_jitter_moves_each_element_by_one_ulp():
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.standard_normal(1000), [0.0, 1.0, -3.0, 1e-30]]).astype(np.float32)
    b = NF.ulp_jitter(a, rng)
    nz = a != 0
    assert np.all(b[~nz] == 0)
    assert np.all(np.abs(b[nz] - a[nz]) == np.spacing(np.abs(a[nz])) * (np.abs(b[nz]) > np.abs(a[nz]))
                  + np.spacing(np.abs(b[nz])) * (np.abs(b[nz]) < np.abs(a[nz])))
    up = (b > a).mean()
    assert 0.4 < up < 0.6


def test_stored_floor_is_reproduced():
    with open(GOLDEN) as f:
        g = json.load(f)
    assert set(g["max"]) == {"all", "geometry", "camera", "attrs_grad"}
    # attributes and upstream gradient alone move the results by about the
    # FP32 rounding of the output; geometry moves them by far more than 1e-5
    assert g["max"]["attrs_grad"]["image_rel"] < 2e-7
    assert g["max"]["geometry"]["image_rel"] > 1e-5
    job = S.config_poses(n_poses=1)[0]
    H = job.camera.height
    rng = np.random.default_rng(2024)
    r = NF.spread(job.scene, job.camera, job.K, np.arange(H * H), job.grad_image.reshape(-1, 3), 2, rng,
                  group="all")
    stored = g["workloads"]["torus4096_128px_C3_K20_pose0"]["all"]
    assert 0.2 * stored["image_rel"] < r["image_rel"] < 5 * stored["image_rel"]
    for n in ("means", "covs", "attrs", "camera"):
        assert 0.1 * stored[n]["inf_over_ref"] < r[n]["inf_over_ref"] < 10 * stored[n]["inf_over_ref"], n
