"""GPU path vs the FP64 oracle, element by element, through the C ABI.

Sizes: the small sphere scene and a ragged 100x72 torus are compared at
every pixel; the 512x512, 10,000-kernel torus (the benchmark workload, in
the launch configuration the benchmark times) on sampled pixels for the
kept sets and at every pixel for the image and the full-image backward
(the oracle blends and differentiates the GPU's own kept sets, so no pixel
is left out: where a near tie or a near-threshold kernel makes more than one
set correct, the difference itself is checked to be one).
"""

import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2205_15401_amd import _native as nat
from paper_2205_15401_amd import render as R
from paper_2205_15401_amd import scenes as S

from parity import check_backward_vs_oracle, check_forward_vs_oracle, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    nat.load()     # fails loudly when the library is missing
    return torch.device("cuda:0")


def gpu_forward(scene, cam, K, eta=0.01):
    m, c, a = to_dev(scene.means), to_dev(scene.covs), to_dev(scene.attrs)
    cs = R.camera_struct(cam)
    img, ws, kept, work = R.render_forward(m, c, a, cs, K, eta, with_wsum=True, with_kept=True)
    st = R.status(work)
    torch.cuda.synchronize()
    H, W = cam.height, cam.width
    return (img.cpu().numpy().reshape(H * W, -1), ws.cpu().numpy().reshape(-1),
            kept.cpu().numpy().reshape(H * W, K), st)


def oracle_forward(scene, cam, K, eta=0.01, pixels=None):
    return O.forward(scene.means, scene.covs, scene.attrs, cam.as_vector(), cam.height, cam.width, K, eta,
                     pixels=pixels)


def check_forward(scene, cam, K, eta=0.01, pixels=None, max_flagged_frac=0.01, name="", full_image=False):
    img, wsum, kept, st = gpu_forward(scene, cam, K, eta)
    own, given = check_forward_vs_oracle(img, wsum, kept, scene, cam, K, eta, pixels, max_flagged_frac,
                                         name=name or f"forward {cam.height}x{cam.width} N={scene.n} K={K}",
                                         full_image=full_image)
    return own, img, kept, st


# ------------------------------------------------------------------ Phi

def test_device_phi_matches_erf():
    from scipy.special import erfc
    x = np.concatenate([np.linspace(-12, 12, 200_001), [0.0, -0.0, 1e-30, -1e-30, 40.0, -40.0]]).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    y = torch.empty_like(xt)
    nat.voge_debug_phi(xt.data_ptr(), y.data_ptr(), x.size, torch.cuda.current_stream().cuda_stream)
    ref = 0.5 * erfc(-x.astype(np.float64))      # accurate in both tails
    err = np.abs(y.cpu().numpy().astype(np.float64) - ref)
    assert err.max() < 2.5e-7, err.max()
    # far tail: relative accuracy is bounded by the rounding of the FP32
    # exponential's argument, about |x|^2 * 2^-24 (x = -8: 4e-6)
    neg = x < -1
    rel = err[neg] / np.maximum(ref[neg], 1e-300)
    keep = ref[neg] > 1e-30
    assert np.all(rel[keep] < 1e-6 + 2e-7 * x[neg][keep].astype(np.float64) ** 2)


# ------------------------------------------------------------- forward

def test_small_spheres_every_pixel():
    job = S.config_small()
    ref, img, kept, st = check_forward(job.scene, job.camera, job.K)
    assert st == 0
    assert (ref.k_eff > 0).mean() > 0.5


def test_ragged_torus_every_pixel():
    rng = np.random.default_rng(12)
    scene = S.torus_scene(rng, 2000, 5, centre=(0.0, 0.0, 3.0))
    cam = S.identity_camera(72, 80.0, height=100)
    check_forward(scene, cam, 20)


@pytest.mark.parametrize("K", [1, 3, 8, 16, 20, 32, 64])
def test_every_k_bucket(K):
    rng = np.random.default_rng(100 + K)
    scene = S.cloud_scene(rng, 1500, 2, std_range=(0.02, 0.08))
    cam = S.identity_camera(48, 48.0, height=40)
    ref, *_ = check_forward(scene, cam, K)
    assert (ref.n_pass > K).any() or K >= 32


def test_rotated_cameras():
    jobs = S.config_poses(n_poses=3, size=96)
    for job in jobs:
        check_forward(job.scene, job.camera, 20)


def test_torus_benchmark_size_sampled_pixels():
    job = S.config_torus()
    rng = np.random.default_rng(22)
    pix = rng.choice(512 * 512, 4000, replace=False)
    ref, *_ = check_forward(job.scene, job.camera, job.K, pixels=pix, full_image=True,
                            name="forward torus10000_512px_C16_K20")
    assert (ref.k_eff == 20).sum() > 1000


def test_eta_values():
    job = S.config_small()
    for eta in (0.1, 0.001):
        check_forward(job.scene, job.camera, 16, eta=eta)


# ---------------------------------------------------------- edge cases

def test_no_kernels_gives_zero_image():
    scene = S.Scene(np.zeros((0, 3), np.float32), np.zeros((0, 6), np.float32), np.zeros((0, 3), np.float32))
    cam = S.identity_camera(33)
    img, wsum, kept, st = gpu_forward(scene, cam, 4)
    assert np.all(img == 0) and np.all(wsum == 0) and np.all(kept == -1) and st == 0


def test_single_kernel_through_centre_is_exp_minus_half():
    cam = S.identity_camera(64, 64.0)
    means = np.array([[1.0, -0.5, 4.0]], np.float32)      # on the ray of pixel (48, 24)
    covs = np.array([[0.05 ** 2, 0, 0, 0.03 ** 2, 0, 0.01 ** 2]], np.float32)
    scene = S.Scene(means, covs, np.ones((1, 1), np.float32))
    img, wsum, kept, st = gpu_forward(scene, cam, 4)
    assert abs(wsum[48 * 64 + 24] - math.exp(-0.5)) < 1e-6
    check_forward(scene, cam, 4)


def test_invalid_kernels_are_skipped_and_reported():
    job = S.config_small()
    sc = job.scene
    covs = sc.covs.copy()
    covs[5, 1] = 1.0                 # not positive definite
    means = sc.means.copy()
    means[9, 0] = np.nan
    scene = S.Scene(means, covs, sc.attrs)
    ref, img, kept, st = check_forward(scene, job.camera, 16)
    assert st & nat.VOGE_STATUS_NOTSPD and st & nat.VOGE_STATUS_NONFINITE
    assert not np.any(kept == 5) and not np.any(kept == 9)
    assert ref.n_invalid == 2


def test_kernels_behind_and_across_the_camera_plane():
    rng = np.random.default_rng(5)
    scene = S.cloud_scene(rng, 600, 3, lo=(-1.5, -1.5, -1.0), hi=(1.5, 1.5, 3.0), std_range=(0.05, 0.3))
    cam = S.identity_camera(40, 40.0)
    check_forward(scene, cam, 12)


def test_principal_point_off_centre_and_nonsquare():
    rng = np.random.default_rng(6)
    scene = S.isotropic_scene(rng, 800, 4)
    cam = S.Camera(R=np.eye(3, dtype=np.float32), T=np.array([0.1, -0.2, 0.3], np.float32), focal=57.5,
                   cx=20.25, cy=31.5, height=61, width=45)
    check_forward(scene, cam, 10)


# ------------------------------------------------------------- backward

def gpu_backward(scene, cam, K, G, eta=0.01, reuse=True):
    """GPU gradients and the kept sets they were taken on (the forward's)."""
    m, c, a = to_dev(scene.means), to_dev(scene.covs), to_dev(scene.attrs)
    cs = R.camera_struct(cam)
    _, _, kept, ws = R.render_forward(m, c, a, cs, K, eta, with_kept=True, for_backward=True)
    gm, gc, ga, gk = R.render_backward(m, c, a, cs, to_dev(G), K, eta, workspace=ws if reuse else None,
                                       reuse=reuse)
    torch.cuda.synchronize()
    kept = kept.cpu().numpy().reshape(-1, K)
    return gm.cpu().numpy(), gc.cpu().numpy(), ga.cpu().numpy(), gk.cpu().numpy(), kept


def check_backward(scene, cam, K, G_full, eta=0.01, reuse=True, name=""):
    """Every pixel's upstream gradient, against the oracle's backward on the
    GPU's kept sets."""
    gm, gc, ga, gk, kept = gpu_backward(scene, cam, K, G_full, eta, reuse)
    C = scene.attrs.shape[1]
    return check_backward_vs_oracle(dict(means=gm, covs=gc, attrs=ga, camera=gk), scene, cam, K,
                                    np.asarray(G_full).reshape(-1, C), kept, eta,
                                    name=name or f"backward {cam.height}x{cam.width} N={scene.n} K={K}")


def test_backward_small_every_pixel():
    job = S.config_small()
    rng = np.random.default_rng(31)
    G = rng.standard_normal((64, 64, 3)).astype(np.float32)
    check_backward(job.scene, job.camera, 16, G)


def test_backward_rotated_camera_ragged():
    job = S.config_poses(n_poses=1, size=72)[0]
    cam = S.Camera(job.camera.R, job.camera.T, 70.0, 33.5, 38.0, 75, 66)
    rng = np.random.default_rng(32)
    G = rng.standard_normal((75, 66, 3)).astype(np.float32)
    check_backward(job.scene, cam, 20, G)


def test_backward_torus_benchmark_size_full_gradient():
    """The 512x512, 10,000-kernel torus with its N(0,1) upstream gradient on
    every pixel: every kernel and camera gradient against the oracle."""
    job = S.config_torus()
    check_backward(job.scene, job.camera, 20, job.grad_image, name="backward torus10000_512px_C16_K20")


def test_backward_without_reuse_matches_reuse():
    job = S.config_small()
    rng = np.random.default_rng(34)
    G = rng.standard_normal((64, 64, 3)).astype(np.float32)
    a = gpu_backward(job.scene, job.camera, 16, G, reuse=True)
    b = gpu_backward(job.scene, job.camera, 16, G, reuse=False)
    for x, y in zip(a[:4], b[:4]):
        np.testing.assert_allclose(x, y, rtol=1e-5, atol=1e-6 * (np.abs(x).max() + 1e-30))


@pytest.mark.parametrize("K", [1, 8, 32, 64])
def test_backward_k_buckets(K):
    rng = np.random.default_rng(200 + K)
    scene = S.cloud_scene(rng, 700, 2, std_range=(0.02, 0.08))
    cam = S.identity_camera(40, 40.0, height=36)
    G = rng.standard_normal((36, 40, 2)).astype(np.float32)
    check_backward(scene, cam, K, G)


def test_autograd_matches_direct_backward():
    job = S.config_small()
    sc = job.scene
    m = to_dev(sc.means).requires_grad_()
    c = to_dev(sc.covs).requires_grad_()
    a = to_dev(sc.attrs).requires_grad_()
    camv = torch.from_numpy(job.camera.as_vector()).requires_grad_()
    img = R.render(m, c, a, camv, K=16, height=64, width=64)
    G = torch.randn_like(img)
    (img * G).sum().backward()
    gm, gc, ga, gk, _ = gpu_backward(sc, job.camera, 16, G.cpu().numpy())
    np.testing.assert_allclose(m.grad.cpu().numpy(), gm, rtol=1e-5, atol=1e-6 * np.abs(gm).max())
    np.testing.assert_allclose(c.grad.cpu().numpy(), gc, rtol=1e-5, atol=1e-6 * np.abs(gc).max())
    np.testing.assert_allclose(a.grad.cpu().numpy(), ga, rtol=1e-5, atol=1e-6 * np.abs(ga).max())
    np.testing.assert_allclose(camv.grad.numpy(), gk, rtol=1e-5, atol=1e-6 * np.abs(gk).max())


def test_autograd_full_covariance_gradient_is_symmetric():
    job = S.config_small()
    sc = job.scene
    full = torch.from_numpy(S.unpack_cov(sc.covs)).cuda().requires_grad_()
    img = R.render(to_dev(sc.means), full, to_dev(sc.attrs), job.camera, K=16)
    img.sum().backward()
    g = full.grad.cpu().numpy()
    np.testing.assert_allclose(g, np.transpose(g, (0, 2, 1)), rtol=0, atol=0)
