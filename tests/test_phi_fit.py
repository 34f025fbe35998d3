"""The device's normal-CDF approximation, checked on the CPU: the
coefficients compiled into trace.hip are the ones phi_fit.py derives, the
argument's scale constants are sqrt(log2 e) and its reciprocal halved, and
the FP32 evaluation (as on the device) stays within 2e-7 of (1 + erf x)/2
everywhere and within a relative bound in the far tail."""

import os
import re

import numpy as np
from scipy.special import erfc

from paper_2205_15401_amd import phi_fit

TRACE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2205_15401_amd", "csrc",
                     "trace.hip")


def horner_coefficients():
    """Coefficients in increasing powers of t, as read from the Horner chain
    fmaf(t, c8, c7), fmaf(t, q, c6), ..., fmaf(t, q, c0)."""
    src = open(TRACE).read()
    body = src[src.index("__device__ __forceinline__ float phi_from"):]
    body = body[:body.index("return")]
    first = re.search(r"fmaf\(t, (-?[\d.e-]+)f, (-?[\d.e-]+)f\)", body)
    rest = re.findall(r"q = fmaf\(t, q, (-?[\d.e-]+)f\)", body)
    c8, c7 = float(first.group(1)), float(first.group(2))
    lower = [float(v) for v in rest]                   # c6, c5, ..., c0
    return np.array(lower[::-1] + [c7, c8], np.float64)


def test_device_coefficients_are_the_fit():
    c = horner_coefficients()
    assert c.size == 9
    fit = (0.5 * phi_fit.fit()).astype(np.float32).astype(np.float64)
    assert np.allclose(c, fit, rtol=1e-6, atol=1e-9), (c, fit)


def scale_constants():
    """SQRT_LOG2E and HALF_OVER_SQRT_LOG2E as compiled into trace.hip."""
    src = open(TRACE).read()
    a = float(re.search(r"SQRT_LOG2E = ([\d.]+)f;", src).group(1))
    b = float(re.search(r"HALF_OVER_SQRT_LOG2E = ([\d.]+)f;", src).group(1))
    return a, b


def test_scale_constants():
    a, b = scale_constants()
    assert abs(a - np.sqrt(np.log2(np.e))) < 1e-8
    assert abs(b - 0.5 / np.sqrt(np.log2(np.e))) < 1e-8


def device_phi(x):
    """Phi as the device evaluates it, in FP32: xs = x sqrt(log2 e),
    e^{-x^2} = 2^{-xs^2}, t = 1/(1 + |xs| / (2 sqrt(log2 e))), Horner in t."""
    c = horner_coefficients().astype(np.float32)
    a, b = (np.float32(v) for v in scale_constants())
    f32 = np.float32
    xs = (x.astype(f32) * a).astype(f32)
    z = np.abs(xs)
    t = (f32(1) / (b * z + f32(1))).astype(f32)
    q = np.full_like(t, c[-1])
    for cc in c[-2::-1]:
        q = (t * q + cc).astype(f32)
    e = np.exp2(-(xs * xs).astype(f32)).astype(f32)
    h = ((t * q).astype(f32) * e).astype(f32)
    return np.where(xs >= 0, f32(1) - h, h).astype(np.float64)


def test_fp32_evaluation_error():
    x = np.linspace(-12, 12, 2_000_001).astype(np.float32)
    phi = device_phi(x)
    ref = 0.5 * erfc(-x.astype(np.float64))
    err = np.abs(phi - ref)
    assert err.max() < 2e-7, err.max()
    neg = x < -1
    rel = err[neg] / np.maximum(ref[neg], 1e-300)
    keep = ref[neg] > 1e-30
    assert np.all(rel[keep] < 1e-6 + 2e-7 * x[neg][keep].astype(np.float64) ** 2)
