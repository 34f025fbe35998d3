"""Multi-view rendering with autograd, and the multi-view shape-fitting loop
of the paper's inverse-rendering experiment (Sec. 4, "Shape Fitting via
Inverse Rendering"): a sphere of Gaussian ellipsoids is fitted to target
views by gradient descent with Adam on the kernel centres and colours, each
iteration on a random subset of the views, with an MSE loss on the RGB
values and on the silhouettes.

The silhouette of a view is the weight sum sum_k W_k of each pixel (Eq. 8
with unit attributes): the renderer draws it as one more attribute channel
fixed at 1, so the image's last channel is the silhouette and its gradient
flows through the same backward as the colours.

Every view subset is one voge_render_batch call for the forward and one
(VOGE_BACKWARD with VOGE_REUSE_PREP, on the forward's workspace) for the
backward.
"""

from __future__ import annotations

from typing import List, Optional, Sequence

import torch

from . import _native as nat
from . import render as R


class Views:
    """A fixed set of cameras of one image size, rendered in any subset."""

    def __init__(self, cameras: Sequence, K: int = 20, eta: float = 0.01):
        if not cameras:
            raise ValueError("no cameras")
        self.cams = [c if isinstance(c, nat.VogeCamera) else R.camera_struct(c) for c in cameras]
        self.height, self.width = self.cams[0].height, self.cams[0].width
        if any(c.height != self.height or c.width != self.width for c in self.cams):
            raise ValueError("all views must have one image size")
        self.K, self.eta = int(K), float(eta)
        self.params = R.params_struct(self.K, self.eta)

    def __len__(self) -> int:
        return len(self.cams)

    def items(self, means, covs, attrs, idx: Sequence[int]):
        arr = (nat.VogeItem * len(idx))()
        N, C = means.shape[0], attrs.shape[1]
        for j, v in enumerate(idx):
            it = arr[j]
            it.means, it.covs, it.attrs = means.data_ptr(), covs.data_ptr(), attrs.data_ptr()
            it.N, it.C = N, C
            it.camera = self.cams[v]
            it.params = self.params
        return arr

    def render(self, means: torch.Tensor, covs: torch.Tensor, attrs: torch.Tensor,
               idx: Optional[Sequence[int]] = None) -> torch.Tensor:
        """Images [len(idx), H, W, C] of the views idx (all by default),
        differentiable w.r.t. means, covs and attrs (gradients summed over
        the views)."""
        idx = list(range(len(self))) if idx is None else [int(i) for i in idx]
        if not idx or any(i < 0 or i >= len(self) for i in idx):
            raise ValueError("bad view indices")
        return _RenderViews.apply(means, covs, attrs, self, tuple(idx))


class _RenderViews(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, covs, attrs, views, idx):
        means, covs, attrs = means.contiguous(), covs.contiguous(), attrs.contiguous()
        R._check_inputs(means, covs, attrs)
        dev = means.device
        V, H, W, C = len(idx), views.height, views.width, attrs.shape[1]
        arr = views.items(means, covs, attrs, idx)
        images = torch.empty((V, H, W, C), dtype=torch.float32, device=dev)
        for j in range(V):
            arr[j].image = images[j].data_ptr()
        nbytes = nat.voge_batch_workspace_size(arr, True)
        ws = R.new_workspace(nbytes, dev)
        nat.voge_render_batch(R.context(dev), arr, nat.VOGE_FORWARD, ws.data_ptr(), nbytes, R._stream(dev))
        ctx.save_for_backward(means, covs, attrs)
        ctx.views, ctx.idx, ctx.ws, ctx.nbytes = views, idx, ws, nbytes
        return images

    @staticmethod
    def backward(ctx, grad_images):
        means, covs, attrs = ctx.saved_tensors
        dev = means.device
        g = grad_images.contiguous()
        V, N, C = len(ctx.idx), means.shape[0], attrs.shape[1]
        gm = torch.empty((V, N, 3), dtype=torch.float32, device=dev)
        gc = torch.empty((V, N, 6), dtype=torch.float32, device=dev)
        ga = torch.empty((V, N, C), dtype=torch.float32, device=dev)
        arr = ctx.views.items(means, covs, attrs, ctx.idx)
        for j in range(V):
            it = arr[j]
            it.grad_image = g[j].data_ptr()
            it.grad_means, it.grad_covs, it.grad_attrs = gm[j].data_ptr(), gc[j].data_ptr(), ga[j].data_ptr()
        nat.voge_render_batch(R.context(dev), arr, nat.VOGE_BACKWARD | nat.VOGE_REUSE_PREP, ctx.ws.data_ptr(),
                              ctx.nbytes, R._stream(dev))
        return gm.sum(0), gc.sum(0), ga.sum(0), None, None


def silhouette_attrs(colors: torch.Tensor) -> torch.Tensor:
    """Colours with the unit channel appended: the rendered image's last
    channel is then the silhouette sum_k W_k."""
    return torch.cat([colors, torch.ones_like(colors[:, :1])], dim=1)


def fit_views(views: Views, means: torch.Tensor, covs: torch.Tensor, colors: torch.Tensor,
              target_rgb: torch.Tensor, target_sil: torch.Tensor, iters: int = 2000, per_iter: int = 5,
              lr_means: float = 0.01, lr_colors: float = 0.05, seed: int = 0):
    """Fit kernel centres and colours to target views (Adam, MSE on RGB and
    silhouette, `per_iter` random views per iteration).  target_rgb is
    [V, H, W, 3], target_sil [V, H, W].  Returns (means, colors, losses) with
    losses a float tensor [iters] on the host."""
    if target_rgb.shape[0] != len(views) or target_sil.shape[0] != len(views):
        raise ValueError("one target per view")
    per_iter = min(int(per_iter), len(views))
    m = means.detach().clone().contiguous().requires_grad_(True)
    c = colors.detach().clone().contiguous().requires_grad_(True)
    cv = covs.detach().contiguous()
    opt = torch.optim.Adam([{"params": [m], "lr": lr_means}, {"params": [c], "lr": lr_colors}])
    gen = torch.Generator().manual_seed(int(seed))
    losses: List[torch.Tensor] = []
    for _ in range(int(iters)):
        idx = torch.randperm(len(views), generator=gen)[:per_iter].tolist()
        img = views.render(m, cv, silhouette_attrs(c), idx)
        sel = torch.tensor(idx, device=target_rgb.device)
        loss = torch.mean((img[..., :3] - target_rgb[sel]) ** 2) + torch.mean((img[..., 3] - target_sil[sel]) ** 2)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        losses.append(loss.detach())
    hist = torch.stack(losses).cpu() if losses else torch.zeros(0)
    return m.detach(), c.detach(), hist
