"""The network kernels evaluate GELU = z Phi(z) with Phi from a Chebyshev fit
of erfc (Press et al., Numerical Recipes, sec. 6.2: erfc(u) = t exp(-u^2 +
P(t)), t = 1 / (1 + u/2)).  These tests read the fit's coefficients from the
kernel source and check them against SciPy's erfc, so a slip in any of them
fails on the CPU: relative error below 1.2e-7 for every u >= 0, and the GELU
built from it, evaluated in float32 as the kernels do, within 2.5e-6 relative
(|z| <= 5) and 4e-7 absolute of the exact GELU."""
import os
import re

import numpy as np
from scipy.special import erfc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_0811_4446_amd", "csrc", "wn_net.hip")


def _coefficients():
    txt = open(SRC).read()
    body = txt[txt.index("half_erfc_fit(float u)"):]
    body = body[:body.index("}")]
    first = re.search(r"float p = ([-+0-9.eE]+)f;", body).group(1)
    rest = re.findall(r"p = fmaf\(p, t, ([-+0-9.eE]+)f\);", body)
    assert len(rest) == 9, rest
    return [float(first)] + [float(c) for c in rest]  # highest power first


def _erfc_fit(u, coef, dtype):
    u = np.asarray(u, dtype=dtype)
    one, half = dtype(1.0), dtype(0.5)
    t = one / (one + half * u)
    p = np.full_like(u, dtype(coef[0]))
    for c in coef[1:]:
        p = p * t + dtype(c)
    return t * np.exp(-u * u + p)


def test_erfc_fit_coefficients_reach_the_published_accuracy():
    coef = _coefficients()
    u = np.linspace(0.0, 12.0, 600001)
    rel = np.abs(_erfc_fit(u, coef, np.float64) / erfc(u) - 1.0)
    assert rel.max() < 1.2e-7, rel.max()


def test_gelu_from_the_fit_in_float32_matches_the_exact_gelu():
    coef = _coefficients()
    z = np.linspace(-10.0, 10.0, 400001).astype(np.float32)
    u = np.abs(z) * np.float32(0.70710678118654752)
    h = np.float32(0.5) * _erfc_fit(u, coef, np.float32)
    phi = np.where(z >= 0, np.float32(1.0) - h, h)
    got = (z * phi).astype(np.float64)
    want = z.astype(np.float64) * 0.5 * erfc(-z.astype(np.float64) / np.sqrt(2.0))
    err = np.abs(got - want)
    assert err.max() < 4e-7, err.max()
    small = np.abs(z) <= 5
    rel = err[small] / np.maximum(np.abs(want[small]), 1e-30)
    assert rel.max() < 2.5e-6, rel.max()
