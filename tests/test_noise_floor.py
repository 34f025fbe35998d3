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
    assert set(g["max"]) == {"all", "geometry", "camera", "attrs_grad", "pairs", "all_with_pairs"}
    # rounding the per-pair derivatives to FP32 moves the gradients by about
    # the FP32 rounding of the output: the inputs set the floor
    for n in ("means", "covs", "attrs", "camera"):
        assert g["max"]["pairs"][n]["inf_over_ref"] < 1e-6, n
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


def test_pair_jitter_moves_each_pair_derivative_by_one_unit_roundoff():
    """The oracle's noise-floor mode on a lone kernel seen by one pixel: the
    attribute gradient W G is moved by exactly one FP32 unit roundoff (2^-24
    relative), up or down as the seed draws; seed 0 is the plain backward
    bit for bit, and one seed always draws the same signs."""
    from oracle import oracle as O
    means = np.array([[0.02, -0.01, 3.0]], np.float32)
    covs = np.array([[0.01, 0.0, 0.0, 0.01, 0.0, 0.01]], np.float32)
    attrs = np.array([[0.5, -2.0]], np.float32)
    cam = S.identity_camera(8, 8.0)
    G = np.array([[1.5, 0.25]])
    pix = [4 * 8 + 4]
    args = (means, covs, attrs, cam.as_vector(), 8, 8, 4, G)
    plain = O.backward(*args, pixels=pix)
    again = O.backward(*args, pixels=pix, jitter_seed=0)
    for n in ("means", "covs", "attrs", "camera"):
        assert np.array_equal(getattr(plain, n), getattr(again, n))
    signs = set()
    for seed in range(1, 9):
        j = O.backward(*args, pixels=pix, jitter_seed=seed)
        rel = (j.attrs / plain.attrs - 1.0) / 2.0 ** -24
        assert np.allclose(rel, rel[0, 0], atol=1e-6) and abs(abs(rel[0, 0]) - 1.0) < 1e-6
        signs.add(int(np.sign(rel[0, 0])))
        j2 = O.backward(*args, pixels=pix, jitter_seed=seed)
        assert np.array_equal(j.attrs, j2.attrs) and np.array_equal(j.covs, j2.covs)
        # the geometric gradients move by a few unit roundoffs at most
        assert np.abs(j.means - plain.means).max() <= 4 * 2.0 ** -24 * np.abs(plain.abs_means).max()
    assert signs == {-1, 1}
