"""Python access to the FP64 CPU oracle (``voge_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg call this module to check and time the GPU library.  The GPU
library never imports it, and it never imports the GPU library.

The oracle follows the VoGE paper step by step (Sec. 3.3, Eq. 3-8; App. A.1-A.3)
in double precision; see the header of ``voge_oracle.c`` for the readings it
takes where the paper is silent.

Algorithmic operation counts (floating-point operations of the method, used to
turn measured time into a fraction of the FP32 vector roofline).  They count
the arithmetic of the formulas as evaluated here, per unit of work:

  FLOP_TRACE = 53 per (ray, passing kernel): S D (9 mul + 6 add), D.SD (5),
      M.SD (5), l = b/a (1), V = M - l D (6), S V (15), V.SV (5), x(-1/2) (1),
      e^q (1), threshold compare not counted.  Only kernels that pass the
      threshold are counted: work on kernels that a coarse stage fails to cull
      is overhead of the implementation, not of the method.
  FLOP_PAIR  = 7 per (ray, kept k, kept m): l_k - l_m, x sqrt(a_m), erf, +1,
      x 1/2, x e^{q_m}, accumulate.
  FLOP_KEPT  = 6 + 2C per (ray, kept kernel): sqrt(a), exp(-E), T e^q, the
      C-channel multiply-add of the blend (2C) and the weight sum (2).
  Backward (given the kept set):
  FLOP_BPAIR = 20 per pair: x (2), Phi (erf, +1, x1/2: 3), Phi' (x^2, exp,
      x 1/sqrt(pi): 3), dm_m += dE_k Phi (2), dE_k m_m Phi' (2), dl_k and dl_m
      updates (4), da_m update (4).
  FLOP_BKEPT = 110 + 4C per kept kernel: G.c_k (2C), W_k G (C), accumulate
      attribute gradient (C), dm, dE (3), dq (1), S V and S D (30), dL/dM (10),
      symmetric dL/dS (40), dL/dD (20), accumulate M and S gradients (9 minus 3
      counted above).  Of these, 2C + 4 (G.c_k, dm, dE, dq) belong with the
      per-pixel pair work and 106 + 2C with the per-kernel chain.
  Exact-integral mode (the quadrature of Eq. 1 for a kept set), per sample
  point t and kept kernel m: FLOP_QUAD_PAIR = 16 -- optical depth term
  (t - l, x sqrt(a), erf, +1, x1/2, x e^q, accumulate: 7) and weight term
  (t - l, square, x a, exp, x sqrt(a/pi), x e^q, x T, x trapezoid weight,
  accumulate: 9); FLOP_QUAD_SAMPLE = 3 per sample point (t, exp(-E), +).
  Sampler (Sec. 3.4, Eq. 10; the kept sets and T given by the forward):
  FLOP_SAMPLE = 2 + 2C per kept kernel: W = T e^q (1), accumulate W phi (2C)
      and W (1); the C divisions per kernel are per-kernel work, not counted.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "voge_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libvoge_oracle.so")
_LOCK = threading.Lock()
_LIB = None

FLAG_TIE = 1
FLAG_ETA = 2

FLOP_TRACE = 53
FLOP_PAIR = 7
FLOP_BPAIR = 20
FLOP_QUAD_PAIR = 16
FLOP_QUAD_SAMPLE = 3


def flop_kept(C: int) -> int:
    return 6 + 2 * C + 2


def flop_sample(C: int) -> int:
    return 2 + 2 * C


def flop_bkept(C: int) -> int:
    return 110 + 4 * C


def flop_bkept_pixel(C: int) -> int:
    return 2 * C + 4


def flop_bkept_chain(C: int) -> int:
    return 106 + 2 * C


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, IEEE semantics, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _lib():
    global _LIB
    with _LOCK:
        if _LIB is None:
            # VOGE_ORACLE_LIB: a build of voge_oracle.c made elsewhere (the
            # sanitizer run of the CPU tests), loaded as it is
            path = os.environ.get("VOGE_ORACLE_LIB")
            if not path:
                build()
                path = _LIB_PATH
            lib = ctypes.CDLL(path)
            P = ctypes.c_void_p
            I = ctypes.c_int
            L = ctypes.c_int64
            Dbl = ctypes.c_double
            lib.oracle_forward.argtypes = [P, P, P, I, I, P, I, I, Dbl, I, P, L, I, P, P, P, P, P, P, P, P, I]
            lib.oracle_forward.restype = I
            lib.oracle_backward.argtypes = [P, P, P, I, I, P, I, I, Dbl, I, P, L, P, I, P, P, P, P, P, P, P, P, I, P, I,
                                            ctypes.c_uint64]
            lib.oracle_backward.restype = I
            lib.oracle_quadrature.argtypes = [P, P, I, P, I, I, Dbl, I, P, L, I, I, P, P, P]
            lib.oracle_quadrature.restype = I
            lib.oracle_transmittance.argtypes = [P, I, P, I, P]
            lib.oracle_transmittance.restype = None
            _LIB = lib
    return _LIB


def _f64(a) -> np.ndarray:
    """Inputs are widened to float64 exactly (float32 arrays lose nothing)."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _pix(pixels, H: int, W: int):
    if pixels is None:
        return None, H * W
    p = np.ascontiguousarray(np.asarray(pixels, dtype=np.int64).reshape(-1))
    if p.size and (p.min() < 0 or p.max() >= H * W):
        raise ValueError("pixel index out of range")
    return p, int(p.size)


class ForwardResult:
    """Per-pixel outputs of the oracle forward (all float64 / int32)."""

    def __init__(self, n, C, K):
        self.image = np.zeros((n, C))
        self.wsum = np.zeros(n)
        self.absum = np.zeros((n, C))
        self.kept_idx = np.full((n, K), -1, np.int32)
        self.kept_rec = np.zeros((n, K, 5))     # l, q, a, E(l_k), W_k
        self.n_pass = np.zeros(n, np.int32)
        self.flags = np.zeros(n, np.int32)
        self.n_invalid = 0

    @property
    def k_eff(self) -> np.ndarray:
        return (self.kept_idx >= 0).sum(axis=1)


def _given(given, n: int, K: int):
    if given is None:
        return None
    g = np.ascontiguousarray(np.asarray(given, np.int32))
    if g.shape != (n, K):
        raise ValueError(f"given kept sets must be ({n}, {K}), got {g.shape}")
    return g


def forward(means, covs, attrs, cam_vec, H: int, W: int, K: int, eta: float = 0.01,
            pixels: Optional[Sequence[int]] = None, threads: int = 0, given=None,
            binned: bool = False) -> ForwardResult:
    """Render the given pixels (linear i*W + j; None = every pixel, row-major).
    given: optional (n_pix, K) kept sets chosen elsewhere (-1 padded); the
    selection (step 4) is then skipped and the blend runs on exactly those
    sets (n_pass = -1, flags = 0).  binned: step 4 on the candidates of
    16x16 screen tiles (same results, less work; a timing mode)."""
    m, c, a, cv = _f64(means), _f64(covs), _f64(attrs), _f64(cam_vec)
    N, C = m.shape[0], a.shape[1]
    assert c.shape == (N, 6) and a.shape[0] == N and cv.size == 15
    pix, n = _pix(pixels, H, W)
    gv = _given(given, n, K)
    r = ForwardResult(n, C, K)
    rc = _lib().oracle_forward(_ptr(m), _ptr(c), _ptr(a), N, C, _ptr(cv), H, W, float(eta), K,
                               _ptr(pix), n, threads, _ptr(r.image), _ptr(r.wsum), _ptr(r.absum),
                               _ptr(r.kept_idx), _ptr(r.kept_rec), _ptr(r.n_pass), _ptr(r.flags), _ptr(gv),
                               int(bool(binned)))
    if rc < 0:
        raise ValueError("oracle_forward: bad arguments")
    r.n_invalid = rc
    return r


class BackwardResult:
    def __init__(self, N, C):
        self.means = np.zeros((N, 3))
        self.covs = np.zeros((N, 6))
        self.attrs = np.zeros((N, C))
        self.camera = np.zeros(15)
        self.abs_means = np.zeros((N, 3))
        self.abs_covs = np.zeros((N, 6))
        self.abs_attrs = np.zeros((N, C))
        self.abs_camera = np.zeros(15)
        self.n_invalid = 0


BLOCK_T = 1      # ablation: no gradient through the transmittance T(l_k)
BLOCK_RHO = 2    # ablation: no gradient through the factor e^{q_k} of Eq. 8


def backward(means, covs, attrs, cam_vec, H: int, W: int, K: int, grad, eta: float = 0.01,
             pixels: Optional[Sequence[int]] = None, threads: int = 0, mode: int = 0,
             given=None, binned: bool = False, jitter_seed: int = 0) -> BackwardResult:
    """Gradients of sum_p <grad_p, C_p> over the given pixels (grad is
    (n_pix, C), or (H, W, C) when pixels is None).  mode: 0, or BLOCK_T and/or
    BLOCK_RHO, the gradient ablations of the paper's pose-estimation ablation
    table ("w/o grad T(r)" and "w/o grad rho(r)").  given: optional (n_pix, K)
    kept sets, as for forward().  jitter_seed: nonzero moves every per-pair
    derivative (dL/dq, dL/dl, dL/da and the pair's weight in the attribute
    gradient) by one FP32 unit roundoff up or down (signs drawn from the seed):
    the noise-floor diagnostic of an implementation that carries them in
    FP32; 0 is the plain backward."""
    m, c, a, cv = _f64(means), _f64(covs), _f64(attrs), _f64(cam_vec)
    N, C = m.shape[0], a.shape[1]
    pix, n = _pix(pixels, H, W)
    gv = _given(given, n, K)
    g = np.ascontiguousarray(np.asarray(grad, np.float64).reshape(n, C))
    r = BackwardResult(N, C)
    rc = _lib().oracle_backward(_ptr(m), _ptr(c), _ptr(a), N, C, _ptr(cv), H, W, float(eta), K,
                                _ptr(pix), n, _ptr(g), threads,
                                _ptr(r.means), _ptr(r.covs), _ptr(r.attrs), _ptr(r.camera),
                                _ptr(r.abs_means), _ptr(r.abs_covs), _ptr(r.abs_attrs), _ptr(r.abs_camera),
                                int(mode), _ptr(gv), int(bool(binned)), int(jitter_seed) & ((1 << 64) - 1))
    if rc < 0:
        raise ValueError("oracle_backward: bad arguments")
    r.n_invalid = rc
    return r


class SampleResult:
    """Per-kernel outputs of the oracle sampler (float64)."""

    def __init__(self, N, C):
        self.num = np.zeros((N, C))       # sum_p W_pk phi_p
        self.den = np.zeros(N)            # sum_p W_pk
        self.alpha = np.zeros((N, C))     # num / den, 0 where den == 0
        self.fwd = None                   # the forward whose kept sets were used


def sample(means, covs, cam_vec, H: int, W: int, K: int, features, eta: float = 0.01,
           threads: int = 0, given=None) -> SampleResult:
    """Inverse reconstruction of Sec. 3.4 (Eq. 10): every kernel takes the
    W-weighted mean of the feature map over the pixels that keep it,
    alpha_k = sum_p W_pk phi_p / sum_p W_pk, with W_pk = T(l_k) e^{q_k} the
    kernel-to-pixel weight of Eq. 8 (the forward's kept records).  features is
    (H, W, C) or (H*W, C).  A kernel that no pixel keeps has den = 0 and is
    given alpha = 0 (the paper does not define the empty quotient).  given:
    optional (H*W, K) kept sets chosen elsewhere, as for forward()."""
    m = _f64(means)
    N = m.shape[0]
    phi = np.asarray(features, np.float64).reshape(H * W, -1)
    C = phi.shape[1]
    fwd = forward(m, covs, np.zeros((N, 1)), cam_vec, H, W, K, eta, threads=threads, given=given)
    r = SampleResult(N, C)
    r.fwd = fwd
    pix, slot = np.nonzero(fwd.kept_idx >= 0)
    k = fwd.kept_idx[pix, slot]
    w = fwd.kept_rec[pix, slot, 4]
    np.add.at(r.num, k, w[:, None] * phi[pix])
    np.add.at(r.den, k, w)
    seen = r.den > 0
    r.alpha[seen] = r.num[seen] / r.den[seen, None]
    return r


def quadrature(means, covs, cam_vec, H: int, W: int, K: int, eta: float = 0.01,
               pixels: Optional[Sequence[int]] = None, n_samples: int = 100_001, threads: int = 0):
    """Exact outer integral of Eq. 1 for each pixel's kept set.
    Returns (w_exact (n,K), w_approx (n,K), total (n,2))."""
    m, c, cv = _f64(means), _f64(covs), _f64(cam_vec)
    N = m.shape[0]
    pix, n = _pix(pixels, H, W)
    we = np.zeros((n, K))
    wa = np.zeros((n, K))
    tot = np.zeros((n, 2))
    rc = _lib().oracle_quadrature(_ptr(m), _ptr(c), N, _ptr(cv), H, W, float(eta), K, _ptr(pix), n,
                                  int(n_samples), threads, _ptr(we), _ptr(wa), _ptr(tot))
    if rc < 0:
        raise ValueError("oracle_quadrature: bad arguments")
    return we, wa, tot


def transmittance(records, t) -> np.ndarray:
    """T(t) = exp(-E(t)) of Eq. 7 for records (n, 3) = (l, q, a)."""
    rec = np.ascontiguousarray(np.asarray(records, np.float64).reshape(-1, 3))
    tt = np.ascontiguousarray(np.asarray(t, np.float64).reshape(-1))
    out = np.zeros(tt.size)
    _lib().oracle_transmittance(_ptr(rec), rec.shape[0], _ptr(tt), tt.size, _ptr(out))
    return out


def forward_flops(n_pass: np.ndarray, k_eff: np.ndarray, C: int) -> int:
    """Algorithmic FLOPs of the forward over a set of rays (see module doc)."""
    kk = k_eff.astype(np.int64)
    return int(FLOP_TRACE * n_pass.astype(np.int64).sum() + FLOP_PAIR * (kk * kk).sum()
               + flop_kept(C) * kk.sum())


def backward_flops(k_eff: np.ndarray, C: int) -> int:
    """Algorithmic FLOPs of the backward proper (kept sets given)."""
    kk = k_eff.astype(np.int64)
    return int(FLOP_BPAIR * (kk * kk).sum() + flop_bkept(C) * kk.sum())
