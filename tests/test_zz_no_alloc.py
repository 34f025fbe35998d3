"""The zero-allocation forward (voge_render_forward_static): the same render
as voge_render_forward with a caller-provided workspace, through the C ABI,
on two calls in a row (the second smaller, so it runs on what the first left
in the library's static workspace), and its size limit checked on the host."""

import numpy as np
import pytest
import torch

from paper_2205_15401_amd import _native as nat
from paper_2205_15401_amd import render as R
from paper_2205_15401_amd import scenes as S

pytestmark = pytest.mark.gpu


def _render_both(dev, scene, cam, K, eta=0.01):
    """(image, wsum, kept) from the workspace entry point and from the static one."""
    m, c, a = (torch.from_numpy(x).to(dev) for x in (scene.means, scene.covs, scene.attrs))
    N, C, H, W = scene.n, scene.channels, cam.height, cam.width
    cs, par = R.camera_struct(cam), R.params_struct(K, eta)
    ctx = R.context(dev)
    s = torch.cuda.current_stream(dev).cuda_stream
    p = lambda t: t.data_ptr()  # noqa: E731
    outs = []
    for static in (False, True):
        img = torch.full((H, W, C), float("nan"), device=dev)
        ws_ = torch.full((H, W), float("nan"), device=dev)
        kept = torch.full((H, W, K), -7, dtype=torch.int32, device=dev)
        if static:
            nat.voge_render_forward_static(ctx, p(m), p(c), p(a), N, C, cs, par, p(img), p(ws_), p(kept), s)
        else:
            wsb = nat.voge_workspace_size(N, C, cs, par, False)
            work = torch.empty(wsb, dtype=torch.uint8, device=dev)
            nat.voge_render_forward(ctx, p(m), p(c), p(a), N, C, cs, par, p(img), p(ws_), p(kept), p(work), wsb, s)
        torch.cuda.synchronize()
        outs.append((img.cpu().numpy(), ws_.cpu().numpy(), kept.cpu().numpy()))
    return outs


def test_static_forward_equals_the_workspace_forward_on_two_calls():
    d = torch.device("cuda:0")
    nat.load()
    rng = np.random.default_rng(77)
    # first call: the 512^2 torus at K = 8 (most of the static workspace);
    # second call: a smaller, ragged rotated render on what the first left
    torus = S.config_torus(with_grad=False)
    cases = [(torus.scene, torus.camera, 8),
             (S.cloud_scene(rng, 3000, 5), S.look_at_camera(np.array([0.4, -0.3, -3.0]), 100), 20)]
    need = [nat.voge_workspace_size(sc.n, sc.channels, R.camera_struct(cam), R.params_struct(K, 0.01), False)
            for sc, cam, K in cases]
    assert need[0] > need[1] and need[0] <= nat.VOGE_STATIC_WORKSPACE_BYTES
    for sc, cam, K in cases:
        (i0, w0, k0), (i1, w1, k1) = _render_both(d, sc, cam, K)
        assert np.isfinite(i0).all() and (k0 >= -1).all()
        np.testing.assert_array_equal(i1, i0)
        np.testing.assert_array_equal(w1, w0)
        np.testing.assert_array_equal(k1, k0)
        assert (k0 >= 0).any()


def test_static_forward_rejects_renders_larger_than_its_workspace():
    d = torch.device("cuda:0")
    nat.load()
    sc = S.config_torus(with_grad=False).scene
    cam = S.identity_camera(1024)
    cs, par = R.camera_struct(cam), R.params_struct(20, 0.01)
    assert nat.voge_workspace_size(sc.n, sc.channels, cs, par, False) > nat.VOGE_STATIC_WORKSPACE_BYTES
    m, c, a = (torch.from_numpy(x).to(d) for x in (sc.means, sc.covs, sc.attrs))
    img = torch.full((1024, 1024, sc.channels), 3.0, device=d)
    with pytest.raises(nat.VogeError) as e:
        nat.voge_render_forward_static(R.context(d), m.data_ptr(), c.data_ptr(), a.data_ptr(), sc.n, sc.channels,
                                       cs, par, img.data_ptr(), None, None, torch.cuda.current_stream(d).cuda_stream)
    assert e.value.code == nat.VOGE_ENOSPACE
    torch.cuda.synchronize()
    assert bool((img == 3.0).all())          # host-checked: outputs untouched
