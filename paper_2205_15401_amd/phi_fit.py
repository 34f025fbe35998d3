"""Coefficients of the device's normal-CDF factor Phi(x) = (1 + erf x)/2.

The device evaluates erfc(z), z = |x|, as

    erfc(z) = t Q(t) e^{-z^2},   t = 1 / (1 + z/2),

with Q a degree-8 polynomial, so that the backward can share e^{-x^2} with
the density Phi'(x) = e^{-x^2}/sqrt(pi).  Q is this project's fit of
e^{z^2} erfc(z) / t (scipy's erfcx) over z in [0, 12]: weighted least
squares on the relative error, reweighted toward equal relative error
(iteratively reweighted least squares, 40 passes).  The fit's relative
error is 4.5e-8 in FP64; evaluated in FP32 (Horner, as on the device),
|Phi - (1 + erf x)/2| < 2e-7 for all x.  The printed coefficients are
Q's times 1/2 (the 1/2 of Phi), in increasing powers of t, as FP32 literals.

Usage: python -m paper_2205_15401_amd.phi_fit
"""

import numpy as np


def fit(deg: int = 8, p: float = 0.5, z_max: float = 12.0, passes: int = 40) -> np.ndarray:
    from scipy.special import erfcx
    z = np.linspace(0.0, z_max, 400001)
    t = 1.0 / (1.0 + p * z)
    f = erfcx(z) / t
    V = np.vander(t, deg + 1, increasing=True)
    w = 1.0 / f
    c = None
    for _ in range(passes):
        c, *_ = np.linalg.lstsq(V * w[:, None], f * w, rcond=None)
        r = (V @ c - f) / f
        w = w * (1.0 + 50.0 * np.abs(r) / np.abs(r).max())
    return c


if __name__ == "__main__":
    c = (0.5 * fit()).astype(np.float32)
    print(", ".join(f"{float(v):.9g}f" for v in c))
