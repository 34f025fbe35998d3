"""ctypes binding of libvoge (include/voge.h, include/voge_debug.h).

Argument marshalling only: every function here calls the C entry point of
the same name.  Pointers are plain integers (device addresses), streams are
hipStream_t handles as integers.  Importing this module does not load the
library; the first call does, and fails loudly when it is not built.
"""

from __future__ import annotations

import ctypes
import os
import threading

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvoge.so")

VOGE_OK = 0
VOGE_EINVAL = -1
VOGE_ENOSPACE = -2
VOGE_EHIP = -3
VOGE_STATUS_NOTSPD = 1
VOGE_STATUS_NONFINITE = 2
VOGE_REUSE_PREP = 1
VOGE_FORWARD = 2
VOGE_BACKWARD = 4
VOGE_GRAPH = 8
VOGE_TUNED = 16
VOGE_SAMPLE = 32
VOGE_BLOCK_T = 64
VOGE_BLOCK_RHO = 128
VOGE_MAX_BATCH = 4096
VOGE_STATIC_WORKSPACE_BYTES = 64 << 20

EXPORTS = [
    "voge_create", "voge_destroy", "voge_workspace_size", "voge_render_forward",
    "voge_render_backward", "voge_status", "voge_last_error", "voge_version", "voge_debug_phi",
    "voge_profile_enable", "voge_profile_read", "voge_batch_workspace_size", "voge_render_batch",
    "voge_batch_status", "voge_tune_batch", "voge_tune_save", "voge_tune_load", "voge_sample",
    "voge_quadrature", "voge_render_forward_static", "voge_debug_bins",
]


class VogeCamera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("T", ctypes.c_float * 3), ("focal", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("height", ctypes.c_int32),
                ("width", ctypes.c_int32)]


class VogeParams(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_float), ("K", ctypes.c_int32)]


class VogeItem(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("covs", ctypes.c_void_p), ("attrs", ctypes.c_void_p),
                ("N", ctypes.c_int32), ("C", ctypes.c_int32), ("camera", VogeCamera), ("params", VogeParams),
                ("image", ctypes.c_void_p), ("wsum", ctypes.c_void_p), ("kept", ctypes.c_void_p),
                ("grad_image", ctypes.c_void_p), ("grad_means", ctypes.c_void_p), ("grad_covs", ctypes.c_void_p),
                ("grad_attrs", ctypes.c_void_p), ("grad_camera", ctypes.c_void_p),
                ("features", ctypes.c_void_p), ("sampled", ctypes.c_void_p), ("sample_weight", ctypes.c_void_p)]


class VogeTuneResult(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("order", ctypes.c_int32), ("bins", ctypes.c_int32),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double)]


class VogePhaseTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("total_ms", ctypes.c_double), ("count", ctypes.c_int64)]


class VogeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libvoge error {code}: {msg}")
        self.code = code


_LOCK = threading.Lock()
_LIB = None


def load(path: str = None):
    """Load libvoge.so and declare its signatures.  VOGE_LIBRARY names another
    build of the same sources (the sanitizer run of the host-side tests)."""
    global _LIB
    with _LOCK:
        if _LIB is not None:
            return _LIB
        if path is None:
            path = os.environ.get("VOGE_LIBRARY") or LIB_PATH
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run `python -m paper_2205_15401_amd.build`")
        lib = ctypes.CDLL(path)
        P, I, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
        CamP, ParP = ctypes.POINTER(VogeCamera), ctypes.POINTER(VogeParams)
        lib.voge_create.argtypes = [ctypes.POINTER(P), I]
        lib.voge_destroy.argtypes = [P]
        lib.voge_workspace_size.argtypes = [I, I, CamP, ParP, I, ctypes.POINTER(SZ)]
        lib.voge_render_forward.argtypes = [P, P, P, P, I, I, CamP, ParP, P, P, P, P, SZ, P]
        lib.voge_render_backward.argtypes = [P, P, P, P, I, I, CamP, ParP, P, P, P, P, P, I, P, SZ, P]
        lib.voge_render_forward_static.argtypes = [P, P, P, P, I, I, CamP, ParP, P, P, P, P]
        lib.voge_sample.argtypes = [P, P, P, I, I, CamP, ParP, P, P, P, I, P, SZ, P]
        lib.voge_quadrature.argtypes = [P, P, P, I, CamP, ParP, I, P, P, P, P, I, P, SZ, P]
        lib.voge_status.argtypes = [P, ctypes.POINTER(ctypes.c_int32), P]
        lib.voge_last_error.argtypes = []
        lib.voge_last_error.restype = ctypes.c_char_p
        lib.voge_version.argtypes = []
        lib.voge_debug_phi.argtypes = [P, P, I, P]
        lib.voge_debug_bins.argtypes = [P, I]
        lib.voge_profile_enable.argtypes = [P, I]
        lib.voge_profile_read.argtypes = [P, ctypes.POINTER(VogePhaseTime), I, ctypes.POINTER(I), I]
        ItemP = ctypes.POINTER(VogeItem)
        lib.voge_batch_workspace_size.argtypes = [ItemP, I, I, ctypes.POINTER(SZ)]
        lib.voge_render_batch.argtypes = [P, ItemP, I, I, P, SZ, P]
        lib.voge_batch_status.argtypes = [P, I, ctypes.POINTER(ctypes.c_int32), P]
        lib.voge_tune_batch.argtypes = [P, ItemP, I, I, P, SZ, P, I, ctypes.POINTER(VogeTuneResult)]
        lib.voge_tune_save.argtypes = [P, ctypes.c_char_p]
        lib.voge_tune_load.argtypes = [P, ctypes.c_char_p]
        for name in EXPORTS:
            if name != "voge_last_error":
                getattr(lib, name).restype = I
        _LIB = lib
        return lib


def voge_last_error() -> str:
    return load().voge_last_error().decode()


def _check(rc: int) -> int:
    if rc != VOGE_OK:
        raise VogeError(rc, voge_last_error())
    return rc


def voge_version() -> int:
    return load().voge_version()


def voge_create(device: int) -> int:
    h = ctypes.c_void_p()
    _check(load().voge_create(ctypes.byref(h), int(device)))
    return h.value


def voge_destroy(ctx: int) -> None:
    _check(load().voge_destroy(ctypes.c_void_p(ctx)))


def voge_workspace_size(N: int, C: int, cam: VogeCamera, params: VogeParams, with_backward: bool) -> int:
    out = ctypes.c_size_t()
    _check(load().voge_workspace_size(int(N), int(C), ctypes.byref(cam), ctypes.byref(params),
                                      int(bool(with_backward)), ctypes.byref(out)))
    return out.value


def voge_render_forward(ctx, means, covs, attrs, N, C, cam, params, image, wsum, kept, workspace,
                        workspace_bytes, stream) -> int:
    return _check(load().voge_render_forward(ctx, means, covs, attrs, int(N), int(C), ctypes.byref(cam),
                                             ctypes.byref(params), image, wsum, kept, workspace,
                                             int(workspace_bytes), stream))


def voge_render_forward_static(ctx, means, covs, attrs, N, C, cam, params, image, wsum, kept, stream) -> int:
    """voge_render_forward with the library's static per-device workspace
    (no workspace argument; allocates nothing)."""
    return _check(load().voge_render_forward_static(ctx, means, covs, attrs, int(N), int(C), ctypes.byref(cam),
                                                    ctypes.byref(params), image, wsum, kept, stream))


def voge_render_backward(ctx, means, covs, attrs, N, C, cam, params, grad_image, grad_means, grad_covs,
                         grad_attrs, grad_camera, flags, workspace, workspace_bytes, stream) -> int:
    return _check(load().voge_render_backward(ctx, means, covs, attrs, int(N), int(C), ctypes.byref(cam),
                                              ctypes.byref(params), grad_image, grad_means, grad_covs,
                                              grad_attrs, grad_camera, int(flags), workspace,
                                              int(workspace_bytes), stream))


def voge_sample(ctx, means, covs, N, C, cam, params, features, sampled, sample_weight, flags, workspace,
                workspace_bytes, stream) -> int:
    return _check(load().voge_sample(ctx, means, covs, int(N), int(C), ctypes.byref(cam), ctypes.byref(params),
                                     features, sampled, sample_weight, int(flags), workspace,
                                     int(workspace_bytes), stream))


def voge_quadrature(ctx, means, covs, N, cam, params, n_samples, w_exact, w_approx, total, kept, flags, workspace,
                    workspace_bytes, stream) -> int:
    return _check(load().voge_quadrature(ctx, means, covs, int(N), ctypes.byref(cam), ctypes.byref(params),
                                         int(n_samples), w_exact, w_approx, total, kept, int(flags), workspace,
                                         int(workspace_bytes), stream))


def voge_status(workspace, stream) -> int:
    st = ctypes.c_int32()
    _check(load().voge_status(workspace, ctypes.byref(st), stream))
    return st.value


def item_array(items):
    """A ctypes array of VogeItem from a sequence of VogeItem."""
    arr = (VogeItem * len(items))()
    for i, it in enumerate(items):
        arr[i] = it
    return arr


def voge_batch_workspace_size(items, with_backward: bool) -> int:
    arr = items if isinstance(items, ctypes.Array) else item_array(items)
    out = ctypes.c_size_t()
    _check(load().voge_batch_workspace_size(arr, len(arr), int(bool(with_backward)), ctypes.byref(out)))
    return out.value


def voge_render_batch(ctx, items, flags, workspace, workspace_bytes, stream) -> int:
    arr = items if isinstance(items, ctypes.Array) else item_array(items)
    return _check(load().voge_render_batch(ctx, arr, len(arr), int(flags), workspace, int(workspace_bytes), stream))


def voge_batch_status(workspace, n_items, stream):
    out = (ctypes.c_int32 * int(n_items))()
    _check(load().voge_batch_status(workspace, int(n_items), out, stream))
    return list(out)


def voge_tune_batch(ctx, items, flags, workspace, workspace_bytes, stream, trials: int = 3) -> VogeTuneResult:
    arr = items if isinstance(items, ctypes.Array) else item_array(items)
    res = VogeTuneResult()
    _check(load().voge_tune_batch(ctx, arr, len(arr), int(flags), workspace, int(workspace_bytes), stream,
                                  int(trials), ctypes.byref(res)))
    return res


def voge_tune_save(ctx, path: str) -> int:
    return _check(load().voge_tune_save(ctx, os.fsencode(path)))


def voge_tune_load(ctx, path: str) -> int:
    return _check(load().voge_tune_load(ctx, os.fsencode(path)))


def voge_debug_phi(x, y, n, stream) -> int:
    return _check(load().voge_debug_phi(x, y, int(n), stream))


def voge_profile_enable(ctx, enable: bool) -> int:
    return _check(load().voge_profile_enable(ctx, int(bool(enable))))


def voge_profile_read(ctx, reset: bool = True):
    """{phase name: (total ms, count)}."""
    arr = (VogePhaseTime * 16)()
    n = ctypes.c_int()
    _check(load().voge_profile_read(ctx, arr, 16, ctypes.byref(n), int(bool(reset))))
    return {arr[i].name.decode(): (arr[i].total_ms, int(arr[i].count)) for i in range(min(n.value, 16))}


def voge_debug_bins(ctx, bins: int) -> int:
    """Coarse-stage bins of untuned calls through ctx: 0 none (the default),
    1 scenes of 16,384 kernels or more, 2 every scene."""
    return _check(load().voge_debug_bins(ctx, int(bins)))
