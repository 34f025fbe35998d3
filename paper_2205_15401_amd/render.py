"""PyTorch front end of libvoge: device tensors in, device tensors out.

PyTorch provides device memory and streams only; every step of the
rendering runs in the library's HIP kernels.  ``render`` is differentiable
w.r.t. means, covariances, attributes and the packed camera vector through a
``torch.autograd.Function`` whose backward calls ``voge_render_backward``.
"""

from __future__ import annotations

import threading
from typing import Dict, Optional, Tuple, Union

import numpy as np
import torch

from . import _native as nat
from .scenes import Camera

_CTX: Dict[int, int] = {}
_CTX_LOCK = threading.Lock()


def context(device: torch.device) -> int:
    """One library context per device, created on first use."""
    idx = device.index if device.index is not None else torch.cuda.current_device()
    with _CTX_LOCK:
        if idx not in _CTX:
            _CTX[idx] = nat.voge_create(idx)
        return _CTX[idx]


def camera_struct(camera: Union[Camera, torch.Tensor, np.ndarray], height: Optional[int] = None,
                  width: Optional[int] = None) -> nat.VogeCamera:
    """A Camera, or a 15-vector (R 9, T 3, F, O_x, O_y) plus height/width."""
    if isinstance(camera, Camera):
        vec = camera.as_vector()
        height, width = camera.height, camera.width
    else:
        t = camera.detach().to("cpu", torch.float32) if isinstance(camera, torch.Tensor) else camera
        vec = np.asarray(t, np.float32).reshape(15)
    if height is None or width is None:
        raise ValueError("height and width are required with a camera vector")
    cs = nat.VogeCamera()
    for e in range(9):
        cs.R[e] = float(vec[e])
    for e in range(3):
        cs.T[e] = float(vec[9 + e])
    cs.focal, cs.cx, cs.cy = float(vec[12]), float(vec[13]), float(vec[14])
    cs.height, cs.width = int(height), int(width)
    return cs


def params_struct(K: int, eta: float) -> nat.VogeParams:
    p = nat.VogeParams()
    p.eta = float(eta)
    p.K = int(K)
    return p


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check_inputs(means, covs, attrs):
    if not (means.is_cuda and covs.is_cuda and attrs.is_cuda):
        raise ValueError("means, covs and attrs must be device tensors")
    for name, t, cols in (("means", means, 3), ("covs", covs, 6)):
        if t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != cols or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 tensor of shape (N, {cols})")
    if attrs.dtype != torch.float32 or attrs.dim() != 2 or not attrs.is_contiguous():
        raise ValueError("attrs must be a contiguous float32 tensor of shape (N, C)")
    if covs.shape[0] != means.shape[0] or attrs.shape[0] != means.shape[0]:
        raise ValueError("means, covs and attrs disagree on N")


def workspace_bytes(N: int, C: int, cam: nat.VogeCamera, params: nat.VogeParams, with_backward: bool) -> int:
    return nat.voge_workspace_size(N, C, cam, params, with_backward)


def new_workspace(nbytes: int, device: torch.device) -> torch.Tensor:
    # torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def render_forward(means: torch.Tensor, covs: torch.Tensor, attrs: torch.Tensor, cam: nat.VogeCamera,
                   K: int = 20, eta: float = 0.01, with_wsum: bool = False, with_kept: bool = False,
                   workspace: Optional[torch.Tensor] = None, for_backward: bool = False):
    """Forward render.  Returns (image [H,W,C], wsum [H,W] or None,
    kept [H,W,K] int32 or None, workspace)."""
    _check_inputs(means, covs, attrs)
    dev = means.device
    N, C = means.shape[0], attrs.shape[1]
    H, W = cam.height, cam.width
    par = params_struct(K, eta)
    need = workspace_bytes(N, C, cam, par, for_backward)
    if workspace is None or workspace.numel() < need:
        workspace = new_workspace(need, dev)
    image = torch.empty((H, W, C), dtype=torch.float32, device=dev)
    wsum = torch.empty((H, W), dtype=torch.float32, device=dev) if with_wsum else None
    kept = torch.empty((H, W, K), dtype=torch.int32, device=dev) if with_kept else None
    nat.voge_render_forward(context(dev), _ptr(means), _ptr(covs), _ptr(attrs), N, C, cam, par,
                            _ptr(image), _ptr(wsum), _ptr(kept), _ptr(workspace), workspace.numel(),
                            _stream(dev))
    return image, wsum, kept, workspace


def render_backward(means: torch.Tensor, covs: torch.Tensor, attrs: torch.Tensor, cam: nat.VogeCamera,
                    grad_image: torch.Tensor, K: int = 20, eta: float = 0.01,
                    workspace: Optional[torch.Tensor] = None, reuse: bool = False, with_camera: bool = True,
                    block_t: bool = False, block_rho: bool = False):
    """Gradients (means [N,3], covs [N,6], attrs [N,C], camera [15] or None).
    block_t / block_rho: the ablated gradients without the path through T or
    through the factor e^q of Eq. 8."""
    _check_inputs(means, covs, attrs)
    dev = means.device
    N, C = means.shape[0], attrs.shape[1]
    par = params_struct(K, eta)
    need = workspace_bytes(N, C, cam, par, True)
    if workspace is None or workspace.numel() < need:
        if reuse:
            raise ValueError("reuse needs the forward's workspace sized for the backward")
        workspace = new_workspace(need, dev)
    g = grad_image.contiguous()
    if g.dtype != torch.float32 or tuple(g.shape) != (cam.height, cam.width, C):
        raise ValueError("grad_image must be float32 of shape (H, W, C)")
    gm = torch.empty((N, 3), dtype=torch.float32, device=dev)
    gc = torch.empty((N, 6), dtype=torch.float32, device=dev)
    ga = torch.empty((N, C), dtype=torch.float32, device=dev)
    gk = torch.empty(15, dtype=torch.float32, device=dev) if with_camera else None
    nat.voge_render_backward(context(dev), _ptr(means), _ptr(covs), _ptr(attrs), N, C, cam, par, _ptr(g),
                             _ptr(gm), _ptr(gc), _ptr(ga), _ptr(gk),
                             (nat.VOGE_REUSE_PREP if reuse else 0) | (nat.VOGE_BLOCK_T if block_t else 0)
                             | (nat.VOGE_BLOCK_RHO if block_rho else 0),
                             _ptr(workspace), workspace.numel(), _stream(dev))
    return gm, gc, ga, gk


def sample(means: torch.Tensor, covs: torch.Tensor, features: torch.Tensor, cam: nat.VogeCamera,
           K: int = 20, eta: float = 0.01, workspace: Optional[torch.Tensor] = None, reuse: bool = False,
           with_weight: bool = False):
    """Sampler of Sec. 3.4 (Eq. 10): features [H,W,C] onto the kernels.
    Returns (alpha [N,C], sum_p W [N] or None, workspace).  ``reuse`` takes
    the kept sets of the last forward on ``workspace`` (same kernels and
    camera)."""
    if not (means.is_cuda and covs.is_cuda and features.is_cuda):
        raise ValueError("means, covs and features must be device tensors")
    for name, t, cols in (("means", means, 3), ("covs", covs, 6)):
        if t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != cols or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 tensor of shape (N, {cols})")
    if covs.shape[0] != means.shape[0]:
        raise ValueError("means and covs disagree on N")
    f = features.contiguous()
    if f.dtype != torch.float32 or f.dim() != 3 or tuple(f.shape[:2]) != (cam.height, cam.width):
        raise ValueError("features must be float32 of shape (H, W, C)")
    dev = means.device
    N, C = means.shape[0], f.shape[2]
    par = params_struct(K, eta)
    need = workspace_bytes(N, C, cam, par, True)
    if workspace is None or workspace.numel() < need:
        if reuse:
            raise ValueError("reuse needs the forward's workspace sized for sampling")
        workspace = new_workspace(need, dev)
    alpha = torch.empty((N, C), dtype=torch.float32, device=dev)
    wk = torch.empty(N, dtype=torch.float32, device=dev) if with_weight else None
    nat.voge_sample(context(dev), _ptr(means), _ptr(covs), N, C, cam, par, _ptr(f), _ptr(alpha), _ptr(wk),
                    nat.VOGE_REUSE_PREP if reuse else 0, _ptr(workspace), workspace.numel(), _stream(dev))
    return alpha, wk, workspace


def quadrature(means: torch.Tensor, covs: torch.Tensor, cam: nat.VogeCamera, K: int = 20, eta: float = 0.01,
               n_samples: int = 4001, workspace: Optional[torch.Tensor] = None, reuse: bool = False):
    """Exact-integral mode: per pixel and kept slot the quadrature weight and
    the closed form (float64 [H,W,K] each), totals [H,W,2] and the kept
    kernels [H,W,K] int32 (voge_quadrature)."""
    for name, t, cols in (("means", means, 3), ("covs", covs, 6)):
        if not t.is_cuda or t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != cols or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 device tensor of shape (N, {cols})")
    dev = means.device
    N = means.shape[0]
    H, W = cam.height, cam.width
    par = params_struct(K, eta)
    need = workspace_bytes(N, 1, cam, par, False)
    if workspace is None or workspace.numel() < need:
        if reuse:
            raise ValueError("reuse needs the forward's workspace")
        workspace = new_workspace(need, dev)
    f64 = dict(dtype=torch.float64, device=dev)
    we, wa = torch.empty((H, W, K), **f64), torch.empty((H, W, K), **f64)
    tot = torch.empty((H, W, 2), **f64)
    kept = torch.empty((H, W, K), dtype=torch.int32, device=dev)
    nat.voge_quadrature(context(dev), _ptr(means), _ptr(covs), N, cam, par, n_samples, _ptr(we), _ptr(wa),
                        _ptr(tot), _ptr(kept), nat.VOGE_REUSE_PREP if reuse else 0, _ptr(workspace),
                        workspace.numel(), _stream(dev))
    return we, wa, tot, kept


def status(workspace: torch.Tensor) -> int:
    """Device status bits of the last forward on this workspace (synchronises)."""
    return nat.voge_status(_ptr(workspace), _stream(workspace.device))


def pack_covariance(cov33: torch.Tensor) -> torch.Tensor:
    """(N,3,3) -> (N,6) packed; off-diagonals average both positions, so the
    gradient w.r.t. the full matrix comes back symmetric."""
    c = cov33
    return torch.stack([c[:, 0, 0], 0.5 * (c[:, 0, 1] + c[:, 1, 0]), 0.5 * (c[:, 0, 2] + c[:, 2, 0]),
                        c[:, 1, 1], 0.5 * (c[:, 1, 2] + c[:, 2, 1]), c[:, 2, 2]], dim=1)


class _Render(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, covs, attrs, cam_vec, height, width, K, eta):
        cam = camera_struct(cam_vec, height, width)
        m, c, a = means.contiguous(), covs.contiguous(), attrs.contiguous()
        image, _, _, ws = render_forward(m, c, a, cam, K, eta, for_backward=True)
        ctx.save_for_backward(m, c, a)
        ctx.cam = cam
        ctx.K, ctx.eta = K, eta
        ctx.ws = ws
        ctx.cam_dtype = cam_vec.dtype if isinstance(cam_vec, torch.Tensor) else None
        return image

    @staticmethod
    def backward(ctx, grad_image):
        m, c, a = ctx.saved_tensors
        gm, gc, ga, gk = render_backward(m, c, a, ctx.cam, grad_image.contiguous().float(), ctx.K, ctx.eta,
                                         workspace=ctx.ws, reuse=True,
                                         with_camera=ctx.needs_input_grad[3])
        ctx.ws = None
        g_cam = None
        if ctx.needs_input_grad[3]:
            g_cam = gk.to("cpu")
        return gm, gc, ga, g_cam, None, None, None, None


def render(means: torch.Tensor, covs: torch.Tensor, attrs: torch.Tensor,
           camera: Union[Camera, torch.Tensor], K: int = 20, eta: float = 0.01,
           height: Optional[int] = None, width: Optional[int] = None) -> torch.Tensor:
    """Differentiable render: image (H, W, C).

    ``covs`` is (N, 6) packed (xx, xy, xz, yy, yz, zz) or (N, 3, 3).
    ``camera`` is a Camera, or a CPU tensor of 15 floats (R, T, F, O_x, O_y)
    with ``height``/``width``; a tensor camera with requires_grad receives
    dL/dcamera."""
    if covs.dim() == 3:
        covs = pack_covariance(covs)
    if isinstance(camera, Camera):
        cam_vec = torch.from_numpy(camera.as_vector())
        height, width = camera.height, camera.width
    else:
        cam_vec = camera
    return _Render.apply(means, covs, attrs, cam_vec, height, width, K, eta)


class Batch:
    """A fixed batch of renders: many cameras and scenes in one call of
    ``voge_render_batch``, with every output and the workspace allocated once.

    ``scenes`` is a list of (means [N,3], covs [N,6], attrs [N,C]) device
    tensors (one entry may serve many items), ``items`` a list of
    (scene index, VogeCamera, K, eta).  ``run`` renders all items; outputs
    live in ``images``, ``wsums``, ``kepts`` and, with a backward, in
    ``grad_means``, ``grad_covs``, ``grad_attrs`` and ``grad_cameras``
    (per item; gradients are per item, not summed over items of one scene).
    With ``sample``, each item also carries a feature map ``features[i]``
    [H,W,C] that ``run(sample=True)`` samples onto the kernels (Sec. 3.4,
    Eq. 10) into ``sampled[i]`` [N,C] and ``sample_weights[i]`` [N].
    """

    def __init__(self, scenes, items, device: torch.device, backward: bool = False, with_wsum: bool = False,
                 with_kept: bool = False, with_camera: bool = False, sample: bool = False):
        for m, c, a in scenes:
            _check_inputs(m, c, a)
        self.device = device
        self.scenes = scenes
        self.n = len(items)
        if not 1 <= self.n <= nat.VOGE_MAX_BATCH:
            raise ValueError(f"a batch holds 1 to {nat.VOGE_MAX_BATCH} items")
        self.backward = backward
        self.sample = sample
        self.arr = (nat.VogeItem * self.n)()
        self.features, self.sampled, self.sample_weights = [], [], []
        self.images, self.wsums, self.kepts = [], [], []
        self.grad_images, self.grad_means, self.grad_covs, self.grad_attrs, self.grad_cameras = [], [], [], [], []
        self.scene_of = []
        f32 = dict(dtype=torch.float32, device=device)
        for i, (si, cam, K, eta) in enumerate(items):
            m, c, a = scenes[si]
            N, C, H, W = m.shape[0], a.shape[1], cam.height, cam.width
            it = self.arr[i]
            it.means, it.covs, it.attrs = _ptr(m), _ptr(c), _ptr(a)
            it.N, it.C = N, C
            it.camera = cam
            it.params = params_struct(K, eta)
            img = torch.empty((H, W, C), **f32)
            self.images.append(img)
            it.image = _ptr(img)
            if with_wsum:
                self.wsums.append(torch.empty((H, W), **f32))
                it.wsum = _ptr(self.wsums[-1])
            if with_kept:
                self.kepts.append(torch.empty((H, W, K), dtype=torch.int32, device=device))
                it.kept = _ptr(self.kepts[-1])
            if backward:
                g = torch.zeros((H, W, C), **f32)
                self.grad_images.append(g)
                it.grad_image = _ptr(g)
                for lst, shape in ((self.grad_means, (N, 3)), (self.grad_covs, (N, 6)), (self.grad_attrs, (N, C))):
                    lst.append(torch.empty(shape, **f32))
                it.grad_means, it.grad_covs, it.grad_attrs = (_ptr(self.grad_means[-1]), _ptr(self.grad_covs[-1]),
                                                              _ptr(self.grad_attrs[-1]))
                if with_camera:
                    self.grad_cameras.append(torch.empty(15, **f32))
                    it.grad_camera = _ptr(self.grad_cameras[-1])
            if sample:
                self.features.append(torch.zeros((H, W, C), **f32))
                self.sampled.append(torch.empty((N, C), **f32))
                self.sample_weights.append(torch.empty(N, **f32))
                it.features, it.sampled, it.sample_weight = (_ptr(self.features[-1]), _ptr(self.sampled[-1]),
                                                             _ptr(self.sample_weights[-1]))
            self.scene_of.append(si)
        self.ws_bytes = nat.voge_batch_workspace_size(self.arr, backward or sample)
        self.workspace = new_workspace(self.ws_bytes, device)

    def set_grad_image(self, i: int, g: torch.Tensor) -> None:
        self.grad_images[i].copy_(g)

    def _flags(self, forward, backward, reuse, sample=False):
        if backward and not self.backward:
            raise ValueError("this batch was built without a backward")
        if sample and not self.sample:
            raise ValueError("this batch was built without sampling")
        flags = (nat.VOGE_FORWARD if forward else 0) | (nat.VOGE_BACKWARD if backward else 0)
        flags |= nat.VOGE_SAMPLE if sample else 0
        return flags | (nat.VOGE_REUSE_PREP if reuse else 0)

    def run(self, forward: bool = True, backward: bool = False, reuse: bool = False, graph: bool = False,
            tuned: bool = False, stream: Optional[int] = None, sample: bool = False, block_t: bool = False,
            block_rho: bool = False) -> None:
        """One call of voge_render_batch on ``stream`` (default: torch's current stream);
        block_t / block_rho: the backward's gradient ablations."""
        flags = self._flags(forward, backward, reuse, sample)
        flags |= (nat.VOGE_BLOCK_T if block_t else 0) | (nat.VOGE_BLOCK_RHO if block_rho else 0)
        flags |= (nat.VOGE_GRAPH if graph else 0) | (nat.VOGE_TUNED if tuned else 0)
        s = _stream(self.device) if stream is None else stream
        nat.voge_render_batch(context(self.device), self.arr, flags, _ptr(self.workspace), self.ws_bytes, s)

    def tune(self, forward: bool = True, backward: bool = False, trials: int = 3,
             stream: Optional[int] = None, sample: bool = False) -> nat.VogeTuneResult:
        """Time the execution choices on this batch (voge_tune_batch); later
        calls of ``run(tuned=True)`` with the same shapes use the fastest."""
        s = _stream(self.device) if stream is None else stream
        return nat.voge_tune_batch(context(self.device), self.arr, self._flags(forward, backward, False, sample),
                                   _ptr(self.workspace), self.ws_bytes, s, trials)

    def status(self):
        """Per-item device status words (synchronises)."""
        return nat.voge_batch_status(_ptr(self.workspace), self.n, _stream(self.device))
