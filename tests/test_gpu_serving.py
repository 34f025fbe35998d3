"""The serving loop on the GPU: requests served in a mix (batched with others,
two batches in flight, admitted under an HBM budget) give the same results as
each request rendered alone, and both match the FP64 oracle."""

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2205_15401_amd import _native as nat
from paper_2205_15401_amd import render as R
from paper_2205_15401_amd import scenes as S
from paper_2205_15401_amd.serving import GpuExecutor, Request, Server, latency_stats, serve_trace

from parity import check_backward_vs_oracle, check_forward_vs_oracle, compare_grad, compare_images, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    nat.load()
    return torch.device("cuda:0")


def test_each_result_is_the_same_alone_and_in_the_mix():
    rng = np.random.default_rng(21)
    scenes = [S.torus_scene(rng, 3000, 3, centre=(0.0, 0.0, 0.0), attr_dist="uniform"),
              S.cloud_scene(rng, 2000, 3, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0))]
    dev = torch.device("cuda:0")
    dscenes = [tuple(to_dev(x) for x in (sc.means, sc.covs, sc.attrs)) for sc in scenes]

    reqs = []
    t = 0.0
    for i in range(16):
        sid = i % 2
        cam = S.random_pose(rng, int(rng.choice([32, 48, 64, 96])))
        bwd = i % 4 in (1, 2)
        sc = scenes[sid]
        H, W = cam.height, cam.width
        G = None
        if bwd:
            G = rng.standard_normal((H, W, 3)).astype(np.float32)
        t += rng.exponential(2e-4)
        reqs.append(Request(scene=sid, camera=cam, backward=bwd, grad_image=G, arrival=t, with_camera=bwd))

    ex = GpuExecutor(dscenes, dev, n_slots=2)
    budget = 3 * max(ex.item_bytes(r) for r in reqs)
    srv = Server(ex, budget, max_batch_items=4)
    serve_trace(srv, reqs)
    torch.cuda.synchronize()
    assert all(r.error is None and r.status == 0 for r in reqs), [r.error for r in reqs]
    assert srv.peak_bytes <= budget
    assert srv.batches < len(reqs)                # some requests shared a batch
    assert latency_stats(reqs)["n"] == len(reqs)

    for r in reqs:
        sc, (m, c, a) = scenes[r.scene], dscenes[r.scene]
        H, W = r.camera.height, r.camera.width
        cs = R.camera_struct(r.camera)
        alone, _, kept, ws = R.render_forward(m, c, a, cs, 20, 0.01, with_kept=True, for_backward=r.backward)
        torch.cuda.synchronize()
        kept = kept.cpu().numpy().reshape(H * W, 20)
        img_mix = r.image.cpu().numpy().reshape(H * W, 3)
        img_alone = alone.cpu().numpy().reshape(H * W, 3)
        # every pixel: the kept sets against the oracle's selection, the images
        # against the oracle's blend of those sets
        own, given = check_forward_vs_oracle(img_mix, None, kept, sc, r.camera, 20, 0.01,
                                             name=f"served request {r.rid}")
        assert compare_images(img_mix, img_alone, given.absum) <= 1.0, f"request {r.rid}: vs alone"
        if not r.backward:
            continue
        gm, gc, ga, gk = R.render_backward(m, c, a, cs, torch.from_numpy(r.grad_image).to(dev), 20, 0.01,
                                           workspace=ws, reuse=True)
        torch.cuda.synchronize()
        mix = dict(means=r.grad_means.cpu().numpy(), covs=r.grad_covs.cpu().numpy(),
                   attrs=r.grad_attrs.cpu().numpy(), camera=r.grad_camera.cpu().numpy())
        check_backward_vs_oracle(mix, sc, r.camera, 20, r.grad_image.reshape(H * W, 3), kept, 0.01,
                                 name=f"served request {r.rid} backward", seed=r.rid)
        bref = O.backward(sc.means, sc.covs, sc.attrs, r.camera.as_vector(), H, W, 20,
                          r.grad_image.reshape(H * W, 3), 0.01, given=kept)
        for name, g_mix, g_alone, av in (("means", r.grad_means, gm, bref.abs_means),
                                         ("covs", r.grad_covs, gc, bref.abs_covs),
                                         ("attrs", r.grad_attrs, ga, bref.abs_attrs),
                                         ("camera", r.grad_camera, gk, bref.abs_camera)):
            elem, inf = compare_grad(g_mix.cpu().numpy(), g_alone.cpu().numpy(), av)
            assert elem <= 1.0 and inf <= 1.0, f"request {r.rid} {name} vs alone: {elem:.3g}, {inf:.3g}"


def test_inputs_made_on_the_caller_stream_and_results_freed_on_completion():
    """Upstream gradients produced by torch work on the caller's stream just
    before submission (behind a long matrix product) are read only once
    ready; each result is reduced on the caller's stream and dropped as soon
    as its request completes, while later batches allocate: every checksum
    equals that of the same request rendered alone afterwards."""
    rng = np.random.default_rng(22)
    dev = torch.device("cuda:0")
    sc = S.torus_scene(rng, 3000, 3, centre=(0.0, 0.0, 0.0), attr_dist="uniform")
    dsc = [tuple(to_dev(x) for x in (sc.means, sc.covs, sc.attrs))]
    cams = [S.random_pose(rng, int(rng.choice([32, 64, 96]))) for _ in range(24)]
    sums = {}

    def on_done(r):
        assert r.error is None, r.error
        vals = [r.image.sum()]
        if r.backward:
            vals += [r.grad_means.abs().sum(), r.grad_covs.abs().sum(), r.grad_attrs.abs().sum()]
        sums[r.rid] = torch.stack(vals)          # computed on the caller's stream
        r.image = r.grad_means = r.grad_covs = r.grad_attrs = None   # freed at once

    ex = GpuExecutor(dsc, dev, n_slots=2)
    srv = Server(ex, 1 << 34, max_batch_items=3, on_done=on_done)
    reqs, seeds = [], []
    big = torch.randn(2048, 2048, device=dev)
    for i, cam in enumerate(cams):
        bwd = i % 2 == 1
        G = None
        if bwd:
            gen = torch.Generator(device=dev)
            gen.manual_seed(1000 + i)
            base = torch.randn((cam.height, cam.width, 3), generator=gen, device=dev)
            busy = (big @ big).sum()                 # keeps the caller's stream busy
            G = base + 0.0 * busy                    # ready only after the product
        r = Request(scene=0, camera=cam, backward=bwd, grad_image=G, arrival=0.0)
        reqs.append(r)
        srv.submit(r)
        srv.pump()
    srv.drain()
    torch.cuda.synchronize()
    assert len(sums) == len(reqs)
    m, c, a = dsc[0]
    for i, r in enumerate(reqs):
        cs = R.camera_struct(r.camera)
        img, _, _, ws = R.render_forward(m, c, a, cs, 20, 0.01, for_backward=r.backward)
        want = [img.sum()]
        if r.backward:
            gen = torch.Generator(device=dev)
            gen.manual_seed(1000 + i)
            G = torch.randn((r.camera.height, r.camera.width, 3), generator=gen, device=dev)
            gm, gc, ga, _ = R.render_backward(m, c, a, cs, G, 20, 0.01, workspace=ws, reuse=True)
            want += [gm.abs().sum(), gc.abs().sum(), ga.abs().sum()]
        torch.testing.assert_close(sums[r.rid], torch.stack(want), rtol=1e-4, atol=1e-6)
