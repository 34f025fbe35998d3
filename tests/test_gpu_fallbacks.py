"""Paths the common workloads never take, forced and checked against the
FP64 oracle through the C ABI, and the largest serving shape.

* Table-full paths.  The backward's tile reduction orders a tile's (pixel,
  kernel) pairs through a hash table of 1,024 kernels in LDS, and the
  sampler accumulates a tile's weights through an LDS table of the same
  size; a kernel that finds its table full sends its pairs to global memory
  one by one.  A scene of small kernels in six depth layers over a 32x32
  image puts 1,250 (K = 20) to 1,700 (K = 64) distinct kept kernels in every
  16x16 tile, so every tile overflows both tables.
* The serving workload's largest request: a 1024x1024 image of the
  200,000-kernel scene, forward and backward with a dense upstream gradient;
  kept sets on sampled pixels, images and every gradient on all pixels.
* The coarse stage's fallbacks: a tile whose bin holds more kernels than
  select sorts in LDS, and tiles past the end of a full pair list, are
  scanned over every record of their item (bins forced on for every scene).
* Bins on and off: the same renders, bit for bit.
"""

import contextlib

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2205_15401_amd import _native as nat
from paper_2205_15401_amd import render as R
from paper_2205_15401_amd import scenes as S

from parity import RTOL, check_backward_vs_oracle, check_forward_vs_oracle, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    nat.load()
    return torch.device("cuda:0")


def layered_scene(seed=5, size=32, layers=6, px_sigma=0.4):
    """One small isotropic kernel near every pixel's ray in each of `layers`
    depth layers (depth U[2,4]); the kernel's screen-space sigma is
    `px_sigma` pixels, so each one is kept by a handful of pixels and a 16x16
    tile keeps well over a thousand distinct kernels."""
    rng = np.random.default_rng(seed)
    F = float(size)
    ii, jj = np.meshgrid(np.arange(size), np.arange(size), indexing="ij")
    pts = []
    for _ in range(layers):
        z = rng.uniform(2.0, 4.0, (size, size))
        di = ii + rng.uniform(-0.3, 0.3, (size, size))
        dj = jj + rng.uniform(-0.3, 0.3, (size, size))
        pts.append(np.stack([(di - size / 2) / F * z, (dj - size / 2) / F * z, z], -1).reshape(-1, 3))
    means = np.concatenate(pts).astype(np.float32)
    sig = px_sigma * means[:, 2] / F
    covs = np.zeros((means.shape[0], 6), np.float32)
    covs[:, 0] = covs[:, 3] = covs[:, 5] = sig ** 2
    attrs = rng.standard_normal((means.shape[0], 3)).astype(np.float32)
    return S.Scene(means, covs, attrs), S.identity_camera(size, F)


def distinct_per_tile(kept, H, W, K):
    k = kept.reshape(H, W, K)
    out = []
    for ti in range(0, H, 16):
        for tj in range(0, W, 16):
            blk = k[ti:ti + 16, tj:tj + 16]
            out.append(len(set(blk[blk >= 0].tolist())))
    return out


@pytest.mark.parametrize("K", [20, 64])
def test_full_tables_backward_matches_the_oracle(K):
    scene, cam = layered_scene()
    H, W = cam.height, cam.width
    rng = np.random.default_rng(60 + K)
    G = rng.standard_normal((H, W, 3)).astype(np.float32)
    m, c, a = to_dev(scene.means), to_dev(scene.covs), to_dev(scene.attrs)
    cs = R.camera_struct(cam)
    img, ws, kept, work = R.render_forward(m, c, a, cs, K, 0.01, with_wsum=True, with_kept=True, for_backward=True)
    gm, gc, ga, gk = R.render_backward(m, c, a, cs, to_dev(G), K, 0.01, workspace=work, reuse=True)
    torch.cuda.synchronize()
    kept = kept.cpu().numpy().reshape(H * W, K)
    assert min(distinct_per_tile(kept, H, W, K)) > 1024, "every tile must overflow the 1,024-entry table"
    check_forward_vs_oracle(img.cpu().numpy(), ws.cpu().numpy(), kept, scene, cam, K,
                            name=f"full tables K={K} forward")
    check_backward_vs_oracle(dict(means=gm.cpu().numpy(), covs=gc.cpu().numpy(), attrs=ga.cpu().numpy(),
                                  camera=gk.cpu().numpy()), scene, cam, K, G.reshape(-1, 3), kept,
                             name=f"full tables K={K} backward")


@pytest.mark.parametrize("K", [20, 64])
def test_full_tables_sampler_matches_the_oracle(K):
    scene, cam = layered_scene(seed=6)
    H, W = cam.height, cam.width
    rng = np.random.default_rng(70 + K)
    phi = rng.standard_normal((H, W, 5)).astype(np.float32)
    m, c, a = to_dev(scene.means), to_dev(scene.covs), to_dev(scene.attrs)
    cs = R.camera_struct(cam)
    # the workspace sized for the sampler's 5 feature channels (the forward's
    # attributes have 3)
    work = R.new_workspace(R.workspace_bytes(scene.n, phi.shape[2], cs, R.params_struct(K, 0.01), True), m.device)
    _, _, kept, work = R.render_forward(m, c, a, cs, K, 0.01, with_kept=True, workspace=work)
    alpha, wk, _ = R.sample(m, c, torch.from_numpy(phi).cuda(), cs, K, 0.01, workspace=work, reuse=True,
                            with_weight=True)
    torch.cuda.synchronize()
    kept = kept.cpu().numpy().reshape(H * W, K)
    assert min(distinct_per_tile(kept, H, W, K)) > 1024
    check_forward_vs_oracle(None, None, kept, scene, cam, K, name=f"full tables K={K} sampler kept sets")
    ref = O.sample(scene.means, scene.covs, cam.as_vector(), H, W, K, phi, 0.01, given=kept)
    absref = O.sample(scene.means, scene.covs, cam.as_vector(), H, W, K, np.abs(phi), 0.01, given=kept)
    al, w = alpha.cpu().numpy().astype(np.float64), wk.cpu().numpy().astype(np.float64)
    seen = ref.den > 0
    assert seen.sum() > 0.5 * scene.n
    assert np.all(al[~seen] == 0.0) and np.all(w[~seen] == 0.0)
    bound = RTOL * (absref.num[seen] / ref.den[seen, None] + np.abs(ref.alpha[seen])) + 1e-30
    ratio = np.abs(al[seen] - ref.alpha[seen]) / bound
    assert ratio.max() <= 1.0, f"alpha, worst {ratio.max():.3g} of the bound"
    wr = np.abs(w[seen] - ref.den[seen]) / (RTOL * ref.den[seen])
    assert wr.max() <= 1.0, f"weight sums, worst {wr.max():.3g} of the bound"


def test_largest_serving_request_matches_the_oracle():
    """1024x1024, the 200,000-kernel scene of the serving workload, a random
    look-at pose, K = 20, forward + backward with a dense N(0,1) upstream
    gradient: kept sets on 2,000 sampled pixels against the oracle's
    selection; image, weight sum and every gradient over all 1,048,576
    pixels against the oracle on the GPU's kept sets."""
    scene = S.serving_scenes(sizes=(10_000, 25_000, 50_000, 100_000, 150_000, 200_000))[5]
    assert scene.n == 200_000
    rng = np.random.default_rng(80)
    cam = S.random_pose(rng, 1024)
    H, W = cam.height, cam.width
    G = rng.standard_normal((H, W, 3)).astype(np.float32)
    m, c, a = to_dev(scene.means), to_dev(scene.covs), to_dev(scene.attrs)
    cs = R.camera_struct(cam)
    img, ws, kept, work = R.render_forward(m, c, a, cs, 20, 0.01, with_wsum=True, with_kept=True, for_backward=True)
    gm, gc, ga, gk = R.render_backward(m, c, a, cs, to_dev(G), 20, 0.01, workspace=work, reuse=True)
    torch.cuda.synchronize()
    assert R.status(work) == 0
    kept = kept.cpu().numpy().reshape(H * W, 20)
    assert (kept[:, 0] >= 0).mean() > 0.2
    pix = np.sort(rng.choice(H * W, 2000, replace=False))
    check_forward_vs_oracle(img.cpu().numpy(), ws.cpu().numpy(), kept, scene, cam, 20, pixels=pix,
                            full_image=True, name="serving 200k 1024px forward")
    check_backward_vs_oracle(dict(means=gm.cpu().numpy(), covs=gc.cpu().numpy(), attrs=ga.cpu().numpy(),
                                  camera=gk.cpu().numpy()), scene, cam, 20, G.reshape(-1, 3), kept,
                             name="serving 200k 1024px backward", floor_draws=2)


def wide_scene(rng, n, sigma, size, centre_z=3.0, spread=0.6, C=3):
    """n isotropic kernels of std `sigma` around (0, 0, centre_z): with sigma
    large enough their eta-ellipsoids reach the camera plane, so their screen
    boxes cover the whole image."""
    means = np.column_stack([rng.uniform(-spread, spread, n), rng.uniform(-spread, spread, n),
                             centre_z + rng.uniform(-0.5, 0.5, n)]).astype(np.float32)
    s = (sigma * rng.uniform(0.8, 1.2, n)).astype(np.float32)
    covs = np.zeros((n, 6), np.float32)
    covs[:, 0] = covs[:, 3] = covs[:, 5] = s ** 2
    return S.Scene(means, covs, rng.standard_normal((n, C)).astype(np.float32))


@contextlib.contextmanager
def bins(mode):
    """Coarse-stage bins of the untuned calls inside: 0 none, 2 every scene."""
    ctx = R.context(torch.device("cuda:0"))
    nat.voge_debug_bins(ctx, mode)
    try:
        yield
    finally:
        nat.voge_debug_bins(ctx, 0)


def check_both(scene, cam, K, name, seed):
    H, W = cam.height, cam.width
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((H, W, scene.attrs.shape[1])).astype(np.float32)
    m, c, a = to_dev(scene.means), to_dev(scene.covs), to_dev(scene.attrs)
    cs = R.camera_struct(cam)
    img, ws, kept, work = R.render_forward(m, c, a, cs, K, 0.01, with_wsum=True, with_kept=True, for_backward=True)
    gm, gc, ga, gk = R.render_backward(m, c, a, cs, to_dev(G), K, 0.01, workspace=work, reuse=True)
    torch.cuda.synchronize()
    kept = kept.cpu().numpy().reshape(H * W, K)
    check_forward_vs_oracle(img.cpu().numpy(), ws.cpu().numpy(), kept, scene, cam, K, name=name + " forward")
    check_backward_vs_oracle(dict(means=gm.cpu().numpy(), covs=gc.cpu().numpy(), attrs=ga.cpu().numpy(),
                                  camera=gk.cpu().numpy()), scene, cam, K, G.reshape(-1, G.shape[2]), kept,
                             name=name + " backward")
    return kept


def test_tiles_with_more_candidates_than_a_bin_holds():
    """Select sorts a tile's bin in LDS when it holds at most 2,048 kernels and
    scans every record of the item otherwise.  2,600 kernels whose boxes
    cover the whole 48x40 image (every tile unbinned) next to the same image
    with a 1,000-kernel scene of small kernels (every tile binned): both
    against the oracle, K = 20 (buffers fill: the early exit is taken)."""
    rng = np.random.default_rng(90)
    wide = wide_scene(rng, 2600, 1.2, 48)
    cam = S.identity_camera(48, 48.0, height=40)
    with bins(2):
        kept = check_both(wide, cam, 20, "unbinned tiles", 91)
        assert (kept >= 0).all()                      # every pixel keeps 20 of the 2,600
        small = S.cloud_scene(rng, 1000, 3, std_range=(0.02, 0.06))
        check_both(small, cam, 20, "binned tiles", 92)


def test_pair_list_overflow_falls_back_per_tile():
    """1,000 kernels whose boxes each cover all 256 tiles of a 256x256 image
    give 256,000 (kernel, tile) pairs, more than the pair list holds (8 per
    kernel + 64 per tile + 1,024 = 25,408): the first tiles are binned, the
    rest scan every record; the whole image against the oracle."""
    rng = np.random.default_rng(93)
    wide = wide_scene(rng, 1000, 1.2, 256, spread=0.8)
    cam = S.identity_camera(256, 256.0)
    with bins(2):
        check_both(wide, cam, 8, "pair-list overflow", 94)


@pytest.mark.parametrize("which", ["torus", "cloud", "poses"])
def test_bins_on_and_off_render_the_same(which):
    """Bins only decide which kernels a tile scans, never what it keeps: the
    same renders with bins for every scene and with none give bit-identical
    images, weight sums and kept sets (512^2 torus of 10,000 kernels; a
    30,000-kernel cloud at 256^2; 16 poses of the
    4,096-kernel torus in one batch), and one of each against the oracle."""
    dev = torch.device("cuda:0")
    if which == "poses":
        jobs = S.config_poses(n_poses=16)
        sc = jobs[0].scene
        dsc = [tuple(to_dev(x) for x in (sc.means, sc.covs, sc.attrs))]
        outs = []
        for mode in (2, 0):
            with bins(mode):
                b = R.Batch(dsc, [(0, R.camera_struct(j.camera), j.K, j.eta) for j in jobs], dev, with_wsum=True,
                            with_kept=True)
                b.run(forward=True)
                torch.cuda.synchronize()
                outs.append([(b.images[i].cpu(), b.wsums[i].cpu(), b.kepts[i].cpu()) for i in range(len(jobs))])
        for (i1, w1, k1), (i2, w2, k2) in zip(*outs):
            assert torch.equal(i1, i2) and torch.equal(w1, w2) and torch.equal(k1, k2)
        j = jobs[3]
        i1, w1, k1 = outs[0][3]
        check_forward_vs_oracle(i1.numpy(), w1.numpy(), k1.numpy().reshape(-1, j.K), sc, j.camera, j.K,
                                name="pose 3 binned")
        return
    if which == "torus":
        job = S.config_torus(with_grad=False)
        scene, cam, K = job.scene, job.camera, job.K
    else:
        rng = np.random.default_rng(95)
        scene = S.cloud_scene(rng, 30_000, 3)
        cam, K = S.identity_camera(256), 16
    m, c, a = to_dev(scene.means), to_dev(scene.covs), to_dev(scene.attrs)
    cs = R.camera_struct(cam)
    outs = []
    for mode in (2, 0):
        with bins(mode):
            img, ws, kept, _ = R.render_forward(m, c, a, cs, K, 0.01, with_wsum=True, with_kept=True)
            torch.cuda.synchronize()
            outs.append((img.cpu(), ws.cpu(), kept.cpu()))
    (i1, w1, k1), (i2, w2, k2) = outs
    assert torch.equal(i1, i2) and torch.equal(w1, w2) and torch.equal(k1, k2)
    H, W = cam.height, cam.width
    pix = np.sort(np.random.default_rng(96).choice(H * W, 3000, replace=False))
    check_forward_vs_oracle(i1.numpy(), w1.numpy(), k1.numpy().reshape(H * W, K), scene, cam, K, pixels=pix,
                            name=f"{which} binned")


def strip_scene(rng, n, focal, width, height, clusters=12):
    """n small isotropic kernels in a few clusters spread along a wide strip
    seen by the identity camera (most 8x8 blocks of the image are empty)."""
    z = rng.uniform(2.0, 4.0, n)
    centre = rng.uniform(-0.45, 0.45, clusters) * width
    col = centre[rng.integers(0, clusters, n)] + rng.normal(0.0, 0.02 * min(width, 2000), n)
    row = rng.uniform(-0.4, 0.4, n) * height
    means = np.column_stack([row * z / focal, col * z / focal, z]).astype(np.float32)   # x: rows, y: columns
    s = rng.uniform(0.005, 0.02, n).astype(np.float32)
    covs = np.zeros((n, 6), np.float32)
    covs[:, 0] = covs[:, 3] = covs[:, 5] = s ** 2
    return S.Scene(means, covs, rng.uniform(0.0, 1.0, (n, 3)).astype(np.float32))


@pytest.mark.parametrize("shape", ["strip", "square"])
def test_block_masks_in_every_cell_mode(shape):
    """Select skips the 8x8 blocks that no kernel's screen box meets, from
    per-item masks counted on a grid of 8x8 cells, of 16x16 tiles when that
    grid would not fit in LDS, and not at all beyond (every block scans).  A
    144x30000 strip (no mask) and a 1040x1040 image (tile cells), each of
    more than 2,048 kernels (the batch size from which masks are built),
    render bit-identically to one batch call over crops of them small enough
    for 8x8 cells (images, weight sums, kept sets), and sampled pixels of the
    large image match the oracle.  The large image is rendered in a batch of
    as many items as the crops (itself and small pads), since the number of
    items sets the depth-bucket resolution of the sort, hence the order of
    equal-bucket kernels and of the blend's sums."""
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(97)
    if shape == "strip":
        H, W, f = 144, 30000, 1000.0
        scene = strip_scene(rng, 2500, f, W, H)
        crops = [(0, o, H, 1000) for o in range(0, W, 1000)]
    else:
        H = W = 1040
        f = 1040.0
        scene = S.cloud_scene(rng, 3000, 3, std_range=(0.005, 0.03))
        crops = [(r, c, 520, 520) for r in (0, 520) for c in (0, 520)]
    cam = S.Camera(R=np.eye(3, dtype=np.float32), T=np.zeros(3, np.float32), focal=f, cx=W / 2.0, cy=H / 2.0,
                   height=H, width=W)
    K = 16
    m, c, a = to_dev(scene.means), to_dev(scene.covs), to_dev(scene.attrs)
    pad = S.Camera(R=cam.R, T=cam.T, focal=f, cx=cam.cx, cy=cam.cy, height=16, width=16)
    full = R.Batch([(m, c, a)], [(0, R.camera_struct(cc), K, 0.01) for cc in [cam] + [pad] * (len(crops) - 1)], dev,
                   with_wsum=True, with_kept=True)
    full.run(forward=True)
    torch.cuda.synchronize()
    img = full.images[0].cpu().numpy().reshape(H, W, 3)
    ws = full.wsums[0].cpu().numpy().reshape(H, W)
    kept = full.kepts[0].cpu().numpy().reshape(H, W, K)
    del full
    assert (kept[..., 0] >= 0).mean() > 0.02
    cams = [S.Camera(R=cam.R, T=cam.T, focal=f, cx=cam.cx - c0, cy=cam.cy - r0, height=h, width=w)
            for (r0, c0, h, w) in crops]
    b = R.Batch([(m, c, a)], [(0, R.camera_struct(cc), K, 0.01) for cc in cams], dev, with_wsum=True,
                with_kept=True)
    b.run(forward=True)
    torch.cuda.synchronize()
    for i, (r0, c0, h, w) in enumerate(crops):
        assert np.array_equal(b.images[i].cpu().numpy().reshape(h, w, 3), img[r0:r0 + h, c0:c0 + w])
        assert np.array_equal(b.wsums[i].cpu().numpy().reshape(h, w), ws[r0:r0 + h, c0:c0 + w])
        assert np.array_equal(b.kepts[i].cpu().numpy().reshape(h, w, K), kept[r0:r0 + h, c0:c0 + w])
    hit = np.flatnonzero(kept.reshape(H * W, K)[:, 0] >= 0)
    pix = np.sort(np.concatenate([rng.choice(hit, 600, replace=False), rng.choice(H * W, 200, replace=False)]))
    check_forward_vs_oracle(img.reshape(H * W, 3), ws.reshape(H * W), kept.reshape(H * W, K), scene, cam, K,
                            pixels=pix, name=f"{shape} block masks")
