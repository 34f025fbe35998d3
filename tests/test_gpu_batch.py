"""Batched rendering (voge_render_batch) vs the FP64 oracle and vs one call
per item, through the C ABI.

Every item of a batch must give what the oracle gives for that item alone,
to the same tolerance as the single-camera tests: kept sets exact up to near
ties (each difference checked to be one), images and weight sums within 1e-5
of the oracle's absolute blend sums, gradients within 1e-5 of the oracle's
per-element absolute sums.  The oracle blends and differentiates the GPU's
own kept sets, so no sampled pixel is left out of any check.
"""

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2205_15401_amd import _native as nat
from paper_2205_15401_amd import render as R
from paper_2205_15401_amd import scenes as S

from parity import check_backward_vs_oracle, check_forward_vs_oracle, compare_grad, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    nat.load()
    return torch.device("cuda:0")


def dev_scene(scene):
    return (to_dev(scene.means), to_dev(scene.covs), to_dev(scene.attrs))


def sparse_gradient(rng, scene, cam, K, eta, n_pix):
    """Upstream gradient non-zero on n_pix sampled pixels; returns (G [H,W,C],
    those pixels, None)."""
    H, W, C = cam.height, cam.width, scene.attrs.shape[1]
    pix = np.sort(rng.choice(H * W, min(n_pix, H * W), replace=False))
    G = np.zeros((H * W, C), np.float32)
    G[pix] = rng.standard_normal((pix.size, C)).astype(np.float32)
    return G.reshape(H, W, C), pix, None


def check_item(batch, i, scene, cam, K, eta, G, pix, fref=None, with_camera=True):
    """Item i of a finished batch against the oracle: kept sets, image and
    weight sum on `pix`, and the backward for the gradient G (non-zero on
    `pix`), all on the GPU's kept sets."""
    H, W, C = cam.height, cam.width, scene.attrs.shape[1]
    img = batch.images[i].cpu().numpy().reshape(H * W, C)
    kept = batch.kepts[i].cpu().numpy().reshape(H * W, K)
    wsum = batch.wsums[i].cpu().numpy().reshape(-1)
    check_forward_vs_oracle(img, wsum, kept, scene, cam, K, eta, pixels=pix, name=f"batch item {i}",
                            full_image=True)
    gpix = np.flatnonzero(np.any(G.reshape(H * W, C) != 0, axis=1))
    grads = dict(means=batch.grad_means[i].cpu().numpy(), covs=batch.grad_covs[i].cpu().numpy(),
                 attrs=batch.grad_attrs[i].cpu().numpy())
    if with_camera:
        grads["camera"] = batch.grad_cameras[i].cpu().numpy()
    return check_backward_vs_oracle(grads, scene, cam, K, G.reshape(H * W, C)[gpix], kept, eta, pixels=gpix,
                                    name=f"batch item {i} backward", seed=i)


def grad_floors(scene, cam, K, eta, G):
    """The oracle's per-element absolute sums for upstream gradient G (the
    tolerance floors of a GPU-vs-GPU gradient comparison)."""
    H, W, C = cam.height, cam.width, scene.attrs.shape[1]
    b = O.backward(scene.means, scene.covs, scene.attrs, cam.as_vector(), H, W, K, G.reshape(H * W, C), eta)
    return b


def assert_grads_close(pairs, bref, what):
    for (g1, g2), a in zip(pairs, (bref.abs_means, bref.abs_covs, bref.abs_attrs, bref.abs_camera)):
        elem, inf = compare_grad(g1.cpu().numpy(), g2.cpu().numpy(), a)
        assert elem <= 1.0 and inf <= 1.0, f"{what}: element {elem:.3g}, inf-norm {inf:.3g}"


def mixed_batch(rng):
    """Scenes and items of mixed sizes, K and eta; one scene shared by two
    items, one item without kernels."""
    spheres = S.config_small().scene
    torus = S.torus_scene(rng, 2000, 5)
    cloud = S.cloud_scene(rng, 1500, 4)
    empty = S.Scene(np.zeros((0, 3), np.float32), np.zeros((0, 6), np.float32), np.zeros((0, 2), np.float32))
    scenes = [spheres, torus, cloud, empty]
    rot = S.look_at_camera(np.array([0.4, -0.3, -0.2]), 72, focal=80.0, target=(0.0, 0.0, 3.0))
    rot.height, rot.cy = 100, 47.5     # ragged tiles, off-centre principal point
    items = [
        (0, S.identity_camera(64), 16, 0.01),
        (1, rot, 20, 0.01),
        (2, S.identity_camera(80, focal=60.0, height=48), 8, 0.01),
        (3, S.identity_camera(16), 4, 0.01),
        (2, S.identity_camera(40), 32, 0.05),
        (0, S.look_at_camera(np.array([0.3, 0.2, -0.5]), 56, focal=50.0, target=(0.0, 0.0, 3.0)), 20, 0.01),
    ]
    return scenes, items


def run_checked_batch(scenes, items, rng, n_pix, with_camera=True):
    dev = torch.device("cuda:0")
    grads, pixs, frefs = [], [], []
    for si, cam, K, eta in items:
        G, pix, fref = sparse_gradient(rng, scenes[si], cam, K, eta, n_pix)
        grads.append(G)
        pixs.append(pix)
        frefs.append(fref)
    dscenes = [dev_scene(sc) for sc in scenes]
    batch = R.Batch(dscenes, [(si, R.camera_struct(cam), K, eta) for si, cam, K, eta in items], dev,
                    backward=True, with_wsum=True, with_kept=True, with_camera=with_camera)
    for i, G in enumerate(grads):
        batch.set_grad_image(i, torch.from_numpy(G))
    batch.run(forward=True, backward=True)
    torch.cuda.synchronize()
    return batch, grads, pixs, frefs, dscenes


def test_mixed_batch_matches_the_oracle_per_item():
    rng = np.random.default_rng(11)
    scenes, items = mixed_batch(rng)
    batch, grads, pixs, frefs, _ = run_checked_batch(scenes, items, rng, n_pix=100_000)
    assert batch.status() == [0] * len(items)
    for i, (si, cam, K, eta) in enumerate(items):
        check_item(batch, i, scenes[si], cam, K, eta, grads[i], pixs[i], frefs[i])
    # the item without kernels renders zeros and a zero camera gradient
    assert float(batch.images[3].abs().max()) == 0.0
    assert float(batch.grad_cameras[3].abs().max()) == 0.0


def test_full_pose_batch_matches_the_oracle():
    """The headline workload as the benchmark runs it: all 256 poses of the
    4,096-kernel torus at 128x128, K = 20, in one forward + backward call with
    each pose's dense N(0,1) upstream gradient.  Kept sets on 256 sampled
    pixels per pose; images, weight sums and every gradient of every pose
    over all of its pixels, on the GPU's kept sets."""
    rng = np.random.default_rng(19)
    jobs = S.config_poses()
    scene = jobs[0].scene
    dev = torch.device("cuda:0")
    ds = dev_scene(scene)
    batch = R.Batch([ds], [(0, R.camera_struct(j.camera), j.K, j.eta) for j in jobs], dev, backward=True,
                    with_wsum=True, with_kept=True, with_camera=True)
    for i, j in enumerate(jobs):
        batch.set_grad_image(i, torch.from_numpy(j.grad_image))
    batch.run(forward=True, backward=True)
    torch.cuda.synchronize()
    assert batch.status() == [0] * len(jobs)
    for i, j in enumerate(jobs):
        H = j.camera.height
        pix = np.sort(rng.choice(H * H, 256, replace=False))
        check_item(batch, i, scene, j.camera, j.K, j.eta, j.grad_image, pix)


def test_pose_batch_matches_the_oracle_and_single_calls():
    """Forty poses of the 4,096-kernel torus at 128x128 (the many-pose
    workload's shapes), one batch; every pose against the oracle on sampled
    pixels and against its own single-camera call on every pixel."""
    rng = np.random.default_rng(12)
    jobs = S.config_poses(n_poses=40)
    scene = jobs[0].scene
    items = [(0, j.camera, j.K, j.eta) for j in jobs]
    batch, grads, pixs, frefs, dscenes = run_checked_batch([scene], items, rng, n_pix=150)
    for i, (_, cam, K, eta) in enumerate(items):
        check_item(batch, i, scene, cam, K, eta, grads[i], pixs[i])
    m, c, a = dscenes[0]
    for i in range(0, len(items), 7):
        _, cam, K, eta = items[i]
        cs = R.camera_struct(cam)
        img, ws, kept, work = R.render_forward(m, c, a, cs, K, eta, with_wsum=True, with_kept=True,
                                               for_backward=True)
        gm, gc, ga, gk = R.render_backward(m, c, a, cs, torch.from_numpy(grads[i]).cuda(), K, eta,
                                           workspace=work, reuse=True)
        torch.cuda.synchronize()
        kb = np.sort(batch.kepts[i].cpu().numpy().reshape(-1, K), axis=1)
        ks = np.sort(kept.cpu().numpy().reshape(-1, K), axis=1)
        same = np.all(kb == ks, axis=1)
        assert same.mean() >= 0.999, f"pose {i}: {np.count_nonzero(~same)} pixels with different kept sets"
        ib, is_ = batch.images[i].cpu().numpy().reshape(-1, 3), img.cpu().numpy().reshape(-1, 3)
        wsb = ws.cpu().numpy().reshape(-1, 1)
        bound = 1e-5 * (np.abs(is_) + wsb * float(np.abs(scene.attrs).max())) + 1e-30
        assert np.all((np.abs(ib - is_) <= bound)[same]), f"pose {i}: batch and single image differ"
        assert_grads_close(((batch.grad_means[i], gm), (batch.grad_covs[i], gc), (batch.grad_attrs[i], ga),
                            (batch.grad_cameras[i], gk)), grad_floors(scene, cam, K, eta, grads[i]),
                           f"pose {i}: batch vs single gradients")


@pytest.mark.parametrize("n_items", [8, 9])
def test_table_upload_paths(n_items):
    """Up to eight item records travel in launch arguments, more through the
    staging ring: both give the single-call images."""
    rng = np.random.default_rng(13)
    scene = S.isotropic_scene(rng, 300)
    dev = torch.device("cuda:0")
    ds = dev_scene(scene)
    cams = [S.random_pose(rng, 32 + 8 * (i % 3), dist_range=(2.5, 3.5)) for i in range(n_items)]
    # the isotropic scene sits around z = 3: shift it to the look-at origin
    m = ds[0] - torch.tensor([0.0, 0.0, 3.0], device=dev)
    ds = (m.contiguous(), ds[1], ds[2])
    batch = R.Batch([ds], [(0, R.camera_struct(c), 12, 0.01) for c in cams], dev, with_kept=True)
    batch.run()
    for i, c in enumerate(cams):
        img, _, kept, _ = R.render_forward(*ds, R.camera_struct(c), 12, 0.01, with_kept=True)
        torch.cuda.synchronize()
        assert torch.equal(torch.sort(kept, dim=2).values, torch.sort(batch.kepts[i], dim=2).values)
        assert torch.allclose(img, batch.images[i], rtol=1e-5, atol=1e-6)


def test_status_words_are_per_item():
    rng = np.random.default_rng(14)
    good = S.isotropic_scene(rng, 64)
    bad = S.isotropic_scene(rng, 64)
    bad.covs[5] = np.array([1.0, 2.0, 0.0, 1.0, 0.0, 1.0], np.float32)   # not positive definite
    bad.means[9, 0] = np.nan
    dev = torch.device("cuda:0")
    cam = R.camera_struct(S.identity_camera(32))
    batch = R.Batch([dev_scene(good), dev_scene(bad)], [(0, cam, 8, 0.01), (1, cam, 8, 0.01), (0, cam, 8, 0.01)],
                    dev)
    batch.run()
    st = batch.status()
    assert st == [0, nat.VOGE_STATUS_NOTSPD | nat.VOGE_STATUS_NONFINITE, 0]
    assert nat.voge_status(batch.workspace.data_ptr(), torch.cuda.current_stream().cuda_stream) == st[1]


def test_forward_then_reuse_backward_equals_one_call():
    """One forward + backward call (the blend and the backward in one kernel,
    k_fwdbwd) against a forward call followed by a backward call that reuses
    its kept sets (k_blend, then k_bwd): the same images bit for bit, and
    gradients within the parity bound (their global sums add in either
    order)."""
    rng = np.random.default_rng(15)
    scenes, items = mixed_batch(rng)
    dev = torch.device("cuda:0")
    dscenes = [dev_scene(sc) for sc in scenes]
    its = [(si, R.camera_struct(cam), K, eta) for si, cam, K, eta in items]
    a = R.Batch(dscenes, its, dev, backward=True, with_camera=True)
    b = R.Batch(dscenes, its, dev, backward=True, with_camera=True)
    Gs = []
    for i, (si, cam, K, eta) in enumerate(items):
        G = rng.standard_normal((cam.height, cam.width, scenes[si].attrs.shape[1])).astype(np.float32)
        Gs.append(G)
        a.set_grad_image(i, torch.from_numpy(G))
        b.set_grad_image(i, torch.from_numpy(G))
    a.run(forward=True, backward=True)
    b.run(forward=True)
    b.run(forward=False, backward=True, reuse=True)
    torch.cuda.synchronize()
    for i, (si, cam, K, eta) in enumerate(items):
        assert torch.equal(a.images[i], b.images[i])
        assert_grads_close(((a.grad_means[i], b.grad_means[i]), (a.grad_covs[i], b.grad_covs[i]),
                            (a.grad_attrs[i], b.grad_attrs[i]), (a.grad_cameras[i], b.grad_cameras[i])),
                           grad_floors(scenes[si], cam, K, eta, Gs[i]), f"item {i}: reuse vs one call")


def test_graph_replays_match_eager_calls():
    """Replays of the cached graph, with eager work and synchronisation in
    between, and after new camera poses of the same shapes, equal eager calls."""
    rng = np.random.default_rng(16)
    jobs = S.config_poses(n_poses=12, size=64, n=2048)
    scene = jobs[0].scene
    dev = torch.device("cuda:0")
    ds = dev_scene(scene)
    its = [(0, R.camera_struct(j.camera), 20, 0.01) for j in jobs]
    eager = R.Batch([ds], its, dev, backward=True, with_camera=True)
    graph = R.Batch([ds], its, dev, backward=True, with_camera=True)
    for i, j in enumerate(jobs):
        eager.set_grad_image(i, torch.from_numpy(j.grad_image))
        graph.set_grad_image(i, torch.from_numpy(j.grad_image))
    side = torch.cuda.Stream()

    def compare(cams):
        for i in range(len(its)):
            assert torch.equal(eager.images[i], graph.images[i]), f"replay image {i}"
            assert_grads_close(((eager.grad_means[i], graph.grad_means[i]), (eager.grad_covs[i], graph.grad_covs[i]),
                                (eager.grad_attrs[i], graph.grad_attrs[i]),
                                (eager.grad_cameras[i], graph.grad_cameras[i])),
                               floors[i] if cams is None else grad_floors(scene, cams[i], 20, 0.01, jobs[i].grad_image),
                               f"replay gradients {i}")

    floors = [grad_floors(scene, j.camera, 20, 0.01, j.grad_image) for j in jobs]

    eager.run(forward=True, backward=True)
    torch.cuda.synchronize()
    for rep in range(3):
        for t in graph.images + graph.grad_means:
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.run(forward=True, backward=True, graph=True, stream=side.cuda_stream)
        side.synchronize()
        x = torch.randn(1 << 20, device=dev).sum()     # eager work between replays
        torch.cuda.synchronize()
        del x
        compare(None)
    # new poses, same shapes: the cached graph renders the new cameras
    new_cams = [S.random_pose(rng, 64) for _ in its]
    for i, c in enumerate(new_cams):
        eager.arr[i].camera = R.camera_struct(c)
        graph.arr[i].camera = R.camera_struct(c)
    eager.run(forward=True, backward=True)
    torch.cuda.synchronize()
    graph.run(forward=True, backward=True, graph=True, stream=side.cuda_stream)
    side.synchronize()
    compare(new_cams)


def test_autotuned_choice_renders_the_same_and_the_cache_round_trips(tmp_path):
    """The tuner times the execution choices on a batch; a tuned call renders
    what the default call renders, and the choices survive a save and load."""
    jobs = S.config_poses(seed=17, n_poses=10, size=64, n=2048)
    scene = jobs[0].scene
    dev = torch.device("cuda:0")
    ds = dev_scene(scene)
    its = [(0, R.camera_struct(j.camera), 20, 0.01) for j in jobs]
    ref = R.Batch([ds], its, dev, backward=True, with_camera=True)
    tuned = R.Batch([ds], its, dev, backward=True, with_camera=True)
    for i, j in enumerate(jobs):
        ref.set_grad_image(i, torch.from_numpy(j.grad_image))
        tuned.set_grad_image(i, torch.from_numpy(j.grad_image))
    side = torch.cuda.Stream()
    ref.run(forward=True, backward=True)
    torch.cuda.synchronize()
    res = tuned.tune(forward=True, backward=True, trials=2, stream=side.cuda_stream)
    assert res.graph in (0, 1) and res.order in (0, 1)
    assert 0 < res.best_ms <= res.default_ms
    for t in tuned.images:
        t.fill_(float("nan"))
    tuned.run(forward=True, backward=True, tuned=True, stream=side.cuda_stream)
    side.synchronize()
    for i, j in enumerate(jobs):
        assert torch.equal(ref.images[i], tuned.images[i])
        assert_grads_close(((ref.grad_means[i], tuned.grad_means[i]), (ref.grad_covs[i], tuned.grad_covs[i]),
                            (ref.grad_attrs[i], tuned.grad_attrs[i]), (ref.grad_cameras[i], tuned.grad_cameras[i])),
                           grad_floors(scene, j.camera, 20, 0.01, j.grad_image), f"tuned item {i}")
    ctx = R.context(dev)
    path = tmp_path / "tune.jsonl"
    nat.voge_tune_save(ctx, str(path))
    lines = path.read_text().splitlines()
    mine = [l for l in lines if "64x64/K20/C3/N12*10" in l]
    assert len(mine) == 1 and '"arch":"gfx' in mine[0]
    assert f'"graph":{res.graph}' in mine[0] and f'"order":{res.order}' in mine[0] and f'"bins":{res.bins}' in mine[0]
    other = tmp_path / "other.jsonl"
    other.write_text('{"arch":"gfx000","key":"k","graph":1,"order":1,"ms":1}\n')
    nat.voge_tune_load(ctx, str(other))                       # another architecture: skipped
    nat.voge_tune_load(ctx, str(path))
    bad = tmp_path / "bad.jsonl"
    bad.write_text('{"arch":"gfx950","key":"k","graph":7,"order":0,"ms":1}\n')
    with pytest.raises(nat.VogeError) as e:
        nat.voge_tune_load(ctx, str(bad))
    assert e.value.code == nat.VOGE_EINVAL
    with pytest.raises(nat.VogeError):
        nat.voge_tune_load(ctx, str(tmp_path / "missing.jsonl"))


def test_uneven_batch_full_size_matches_the_oracle():
    """The uneven batch at its full size in one call: 64 cloud scenes of
    1,000-100,000 kernels, 64^2-512^2 images, K in {8, 16, 32} (three K-buffer
    groups), forward + backward; every item against the oracle on 64 sampled
    pixels and through an upstream gradient on those pixels."""
    rng = np.random.default_rng(31)
    jobs = S.config_uneven()
    scenes = [j.scene for j in jobs]
    items = [(i, j.camera, j.K, j.eta) for i, j in enumerate(jobs)]
    batch, grads, pixs, frefs, _ = run_checked_batch(scenes, items, rng, n_pix=64)
    assert batch.status() == [0] * len(items)
    for i, (si, cam, K, eta) in enumerate(items):
        check_item(batch, i, scenes[si], cam, K, eta, grads[i], pixs[i], frefs[i])


def test_repeated_calls_are_deterministic():
    """Two identical calls: images, weight sums and kept lists bit for bit;
    gradients (float atomics in any order) within the oracle's floors."""
    rng = np.random.default_rng(41)
    scenes, items = mixed_batch(rng)
    dev = torch.device("cuda:0")
    dscenes = [dev_scene(sc) for sc in scenes]
    its = [(si, R.camera_struct(cam), K, eta) for si, cam, K, eta in items]
    runs = []
    Gs = [rng.standard_normal((cam.height, cam.width, scenes[si].attrs.shape[1])).astype(np.float32)
          for si, cam, K, eta in items]
    for _ in range(2):
        b = R.Batch(dscenes, its, dev, backward=True, with_wsum=True, with_kept=True, with_camera=True)
        for i, G in enumerate(Gs):
            b.set_grad_image(i, torch.from_numpy(G))
        b.run(forward=True, backward=True)
        torch.cuda.synchronize()
        runs.append(b)
    a, b = runs
    for i, (si, cam, K, eta) in enumerate(items):
        assert torch.equal(a.images[i], b.images[i]) and torch.equal(a.wsums[i], b.wsums[i])
        assert torch.equal(a.kepts[i], b.kepts[i])
        assert_grads_close(((a.grad_means[i], b.grad_means[i]), (a.grad_covs[i], b.grad_covs[i]),
                            (a.grad_attrs[i], b.grad_attrs[i]), (a.grad_cameras[i], b.grad_cameras[i])),
                           grad_floors(scenes[si], cam, K, eta, Gs[i]), f"item {i}: repeat")


def test_channel_counts_through_both_attribute_paths():
    """C = 1 and 64 and 1024 (the maximum) and 4: attribute gathers take the
    four-channel path when C is a multiple of 4, the scalar path otherwise,
    and the backward reduction makes one pass per 8 channels."""
    rng = np.random.default_rng(42)
    scenes, items = [], []
    for C, size in ((1, 40), (4, 32), (64, 24), (1024, 16)):
        sc = S.isotropic_scene(rng, 200, C)
        sc.attrs = rng.standard_normal((200, C)).astype(np.float32)
        scenes.append(sc)
        items.append((len(scenes) - 1, S.identity_camera(size), 12, 0.01))
    batch, grads, pixs, frefs, _ = run_checked_batch(scenes, items, rng, n_pix=100_000)
    for i, (si, cam, K, eta) in enumerate(items):
        check_item(batch, i, scenes[si], cam, K, eta, grads[i], pixs[i], frefs[i])


def test_gradient_staging_on_and_off_match_the_oracle():
    """The backward's tile reduction stages the upstream gradient in LDS when
    every item of a K-buffer group has at most 4 channels, and reads it from
    global memory otherwise: the same 3-channel item alone (staged) and next
    to a 5-channel item with the same K (not staged) both match the oracle
    and each other."""
    rng = np.random.default_rng(77)
    three = S.torus_scene(rng, 1800, 3, centre=(0.0, 0.0, 3.0))
    five = S.cloud_scene(rng, 900, 5)
    cam3 = S.identity_camera(56, focal=60.0, height=40)
    cam5 = S.identity_camera(32)
    alone, g_a, p_a, f_a, _ = run_checked_batch([three], [(0, cam3, 20, 0.01)], rng, n_pix=100_000)
    check_item(alone, 0, three, cam3, 20, 0.01, g_a[0], p_a[0], f_a[0])
    dev = torch.device("cuda:0")
    mixed = R.Batch([dev_scene(three), dev_scene(five)],
                    [(0, R.camera_struct(cam3), 20, 0.01), (1, R.camera_struct(cam5), 20, 0.01)], dev,
                    backward=True, with_wsum=True, with_kept=True, with_camera=True)
    G5, _, _ = sparse_gradient(rng, five, cam5, 20, 0.01, 100_000)
    mixed.set_grad_image(0, torch.from_numpy(g_a[0]))
    mixed.set_grad_image(1, torch.from_numpy(G5))
    mixed.run(forward=True, backward=True)
    torch.cuda.synchronize()
    check_item(mixed, 0, three, cam3, 20, 0.01, g_a[0], p_a[0], f_a[0])
    bref = grad_floors(three, cam3, 20, 0.01, g_a[0])
    assert_grads_close([(alone.grad_means[0], mixed.grad_means[0]), (alone.grad_covs[0], mixed.grad_covs[0]),
                        (alone.grad_attrs[0], mixed.grad_attrs[0]), (alone.grad_cameras[0], mixed.grad_cameras[0])],
                       bref, "staged vs global upstream gradient")


def test_device_calls_reject_bad_workspaces_and_pointers():
    dev = torch.device("cuda:0")
    ctx = R.context(dev)
    sc = S.config_small().scene
    m, c, a = dev_scene(sc)
    cs = R.camera_struct(S.identity_camera(32))
    it = nat.VogeItem()
    it.means, it.covs, it.attrs = m.data_ptr(), c.data_ptr(), a.data_ptr()
    it.N, it.C = sc.n, 3
    it.camera = cs
    it.params = R.params_struct(8, 0.01)
    img = torch.empty((32, 32, 3), device=dev)
    it.image = img.data_ptr()
    need = nat.voge_batch_workspace_size([it], False)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    with pytest.raises(nat.VogeError) as e:
        nat.voge_render_batch(ctx, [it], nat.VOGE_FORWARD, ws.data_ptr(), need - 256, s)
    assert e.value.code == nat.VOGE_ENOSPACE
    with pytest.raises(nat.VogeError) as e:
        nat.voge_render_batch(ctx, [it], nat.VOGE_BACKWARD, ws.data_ptr(), need, s)   # no gradient pointers
    assert e.value.code == nat.VOGE_EINVAL
    nat.voge_render_batch(ctx, [it], nat.VOGE_FORWARD, ws.data_ptr(), need, s)
    torch.cuda.synchronize()
    assert torch.isfinite(img).all()
