"""The device's normal-CDF approximation, checked on the CPU: the
coefficients compiled into trace.hip are the ones phi_fit.py derives, and
their FP32 Horner evaluation (as on the device) stays within 2e-7 of
(1 + erf x)/2 everywhere and within a relative bound in the far tail."""

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


def test_fp32_evaluation_error():
    c = horner_coefficients().astype(np.float32)
    f32 = np.float32
    x = np.linspace(-12, 12, 2_000_001).astype(f32)
    z = np.abs(x)
    t = (f32(1) / (f32(0.5) * z + f32(1))).astype(f32)
    q = np.full_like(t, c[-1])
    for cc in c[-2::-1]:
        q = (t * q + cc).astype(f32)
    e = np.exp(-(x * x).astype(f32)).astype(f32)
    h = ((t * q).astype(f32) * e).astype(f32)
    phi = np.where(x >= 0, f32(1) - h, h).astype(np.float64)
    ref = 0.5 * erfc(-x.astype(np.float64))
    err = np.abs(phi - ref)
    assert err.max() < 2e-7, err.max()
    neg = x < -1
    rel = err[neg] / np.maximum(ref[neg], 1e-300)
    keep = ref[neg] > 1e-30
    assert np.all(rel[keep] < 1e-6 + 2e-7 * x[neg][keep].astype(np.float64) ** 2)
