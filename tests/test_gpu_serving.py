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

from parity import compare_grad, compare_images, to_dev

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

    reqs, refs = [], []
    t = 0.0
    for i in range(16):
        sid = i % 2
        cam = S.random_pose(rng, int(rng.choice([32, 48, 64, 96])))
        bwd = i % 4 in (1, 2)
        sc = scenes[sid]
        H, W = cam.height, cam.width
        ref = O.forward(sc.means, sc.covs, sc.attrs, cam.as_vector(), H, W, 20, 0.01)
        G = None
        if bwd:
            G = rng.standard_normal((H * W, 3)).astype(np.float32)
            G[ref.flags != 0] = 0.0               # no gradient through near ties
            G = G.reshape(H, W, 3)
        t += rng.exponential(2e-4)
        reqs.append(Request(scene=sid, camera=cam, backward=bwd, grad_image=G, arrival=t, with_camera=bwd))
        refs.append(ref)

    ex = GpuExecutor(dscenes, dev, n_slots=2)
    budget = 3 * max(ex.item_bytes(r) for r in reqs)
    srv = Server(ex, budget, max_batch_items=4)
    serve_trace(srv, reqs)
    torch.cuda.synchronize()
    assert all(r.error is None and r.status == 0 for r in reqs), [r.error for r in reqs]
    assert srv.peak_bytes <= budget
    assert srv.batches < len(reqs)                # some requests shared a batch
    assert latency_stats(reqs)["n"] == len(reqs)

    for r, ref in zip(reqs, refs):
        sc, (m, c, a) = scenes[r.scene], dscenes[r.scene]
        H, W = r.camera.height, r.camera.width
        cs = R.camera_struct(r.camera)
        alone, _, _, ws = R.render_forward(m, c, a, cs, 20, 0.01, for_backward=r.backward)
        torch.cuda.synchronize()
        same = ref.flags == 0
        img_mix = r.image.cpu().numpy().reshape(H * W, 3)
        img_alone = alone.cpu().numpy().reshape(H * W, 3)
        assert compare_images(img_mix, ref.image, ref.absum, mask=same) <= 1.0, f"request {r.rid}: vs oracle"
        assert compare_images(img_mix, img_alone, ref.absum, mask=same) <= 1.0, f"request {r.rid}: vs alone"
        if not r.backward:
            continue
        gm, gc, ga, gk = R.render_backward(m, c, a, cs, torch.from_numpy(r.grad_image).to(dev), 20, 0.01,
                                           workspace=ws, reuse=True)
        torch.cuda.synchronize()
        bref = O.backward(sc.means, sc.covs, sc.attrs, r.camera.as_vector(), H, W, 20,
                          r.grad_image.reshape(H * W, 3), 0.01)
        for name, g_mix, g_alone, rv, av in (("means", r.grad_means, gm, bref.means, bref.abs_means),
                                             ("covs", r.grad_covs, gc, bref.covs, bref.abs_covs),
                                             ("attrs", r.grad_attrs, ga, bref.attrs, bref.abs_attrs),
                                             ("camera", r.grad_camera, gk, bref.camera, bref.abs_camera)):
            for what, other in (("oracle", rv), ("alone", g_alone.cpu().numpy())):
                elem, inf = compare_grad(g_mix.cpu().numpy(), other, av)
                assert elem <= 1.0 and inf <= 1.0, f"request {r.rid} {name} vs {what}: {elem:.3g}, {inf:.3g}"
