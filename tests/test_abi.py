"""The C-ABI library loads, exports every symbol its headers declare, and
rejects bad arguments on the host (no GPU work is issued by these tests)."""

import ctypes
import glob
import os
import re

import pytest

from paper_2205_15401_amd import _native as nat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b(voge_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(nat.LIB_PATH):
        pytest.fail("libvoge.so is not built (run python -m paper_2205_15401_amd.build)")
    return nat.load()


def test_headers_declare_the_entry_points():
    names = declared_symbols()
    assert {"voge_create", "voge_destroy", "voge_workspace_size", "voge_render_forward",
            "voge_render_backward", "voge_status", "voge_last_error", "voge_version"} <= names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(nat.EXPORTS) >= declared_symbols()


def test_version(lib):
    assert nat.voge_version() == 10000


def cam(h=64, w=64, f=64.0):
    c = nat.VogeCamera()
    c.R[0] = c.R[4] = c.R[8] = 1.0
    c.focal, c.cx, c.cy, c.height, c.width = f, w / 2, h / 2, h, w
    return c


def par(K=20, eta=0.01):
    p = nat.VogeParams()
    p.K, p.eta = K, eta
    return p


def test_workspace_size_grows_with_problem(lib):
    a = nat.voge_workspace_size(100, 3, cam(), par(), False)
    b = nat.voge_workspace_size(100, 3, cam(), par(), True)
    c = nat.voge_workspace_size(10_000, 3, cam(), par(), False)
    d = nat.voge_workspace_size(100, 3, cam(512, 512, 512.0), par(), False)
    assert 0 < a < b and a < c and a < d
    assert nat.voge_workspace_size(0, 1, cam(), par(1), False) > 0


@pytest.mark.parametrize("args, what", [
    (dict(N=-1), "N"), (dict(C=0), "C"), (dict(C=2000), "C"), (dict(K=0), "K"), (dict(K=65), "K"),
    (dict(h=0), "image"), (dict(w=40000), "image"), (dict(f=0.0), "focal"), (dict(f=float("nan")), "focal"),
])
def test_workspace_size_rejects_bad_arguments(lib, args, what):
    N, C, K = args.get("N", 10), args.get("C", 3), args.get("K", 20)
    c = cam(args.get("h", 64), args.get("w", 64), args.get("f", 64.0))
    with pytest.raises(nat.VogeError) as e:
        nat.voge_workspace_size(N, C, c, par(K), True)
    assert e.value.code == nat.VOGE_EINVAL
    assert what.lower() in nat.voge_last_error().lower() or what == "image"


def test_calls_without_context_are_rejected_on_the_host(lib):
    with pytest.raises(nat.VogeError) as e:
        nat.voge_render_forward(None, None, None, None, 0, 3, cam(), par(), None, None, None, None, 0, None)
    assert e.value.code == nat.VOGE_EINVAL
    with pytest.raises(nat.VogeError) as e:
        nat.voge_render_backward(None, None, None, None, 0, 3, cam(), par(), None, None, None, None, None, 0,
                                 None, 0, None)
    assert e.value.code == nat.VOGE_EINVAL
    with pytest.raises(nat.VogeError):
        nat.voge_status(None, None)
    with pytest.raises(nat.VogeError):
        nat.voge_debug_phi(None, None, 5, None)
    with pytest.raises(nat.VogeError):
        nat.voge_create(-1)


def test_bad_eta_is_rejected_before_any_device_work(lib):
    # a non-null fake context: argument checks run before the context is used
    fake_ctx = ctypes.c_void_p(1).value
    for eta in (0.0, 1.0, -0.5, float("nan")):
        with pytest.raises(nat.VogeError) as e:
            nat.voge_render_forward(fake_ctx, None, None, None, 0, 3, cam(), par(20, eta), 1, None, None, 256,
                                    1 << 20, None)
        assert e.value.code == nat.VOGE_EINVAL
