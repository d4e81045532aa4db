"""The GELU of the library's BF16 and FP8 paths (gelu_fast in csrc/common.h: z sigma(g(z)) with g
an odd quintic fitted to the normal CDF) evaluated on the CPU with the constants read from the
source, in FP32 arithmetic step by step as the kernel does, against the exact erf GELU: the error
bounds its comment and the header state hold on the whole real line."""
import os
import re

import numpy as np
from scipy.special import erf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _constants():
    src = open(os.path.join(ROOT, "paper_2601_17554_amd", "csrc", "common.h")).read()
    body = src[src.index("float gelu_fast(float z)"):]
    body = body[:body.index("\n}")]
    k5, k3 = map(float, re.search(r"fmaf\(z2, ([-0-9.e]+)f, ([-0-9.e]+)f\)", body).groups())
    k1 = float(re.search(r"fmaf\(p, z2, ([-0-9.e]+)f\)", body).group(1))
    clamp = float(re.search(r"fmaxf\(z, -([0-9.]+)f\)", body).group(1))
    return np.float32(k1), np.float32(k3), np.float32(k5), np.float32(clamp)


def gelu_fast(z):
    k1, k3, k5, clamp = _constants()
    z = z.astype(np.float32)
    zc = np.clip(z, -clamp, clamp).astype(np.float32)
    z2 = (zc * zc).astype(np.float32)
    p = (z2.astype(np.float64) * k5 + k3).astype(np.float32)   # fma: one rounding
    p = (p.astype(np.float64) * z2 + k1).astype(np.float32)
    g = (zc * p).astype(np.float32)
    e = np.exp2(g.astype(np.float64)).astype(np.float32)
    r = (1.0 / (np.float32(1.0) + e).astype(np.float64)).astype(np.float32)
    return (z * r).astype(np.float32), r


def test_gelu_fast_error_bounds():
    z = np.linspace(-40.0, 40.0, 4_000_001)  # (and |z| up to 1e6: the value at -10 times z)
    g, cdf = gelu_fast(z)
    z32 = z.astype(np.float32).astype(np.float64)
    phi = 0.5 * (1.0 + erf(z32 / np.sqrt(2.0)))
    assert np.max(np.abs(cdf - phi)) <= 1.9e-5
    assert np.max(np.abs(g - z32 * phi)) <= 5.5e-5


def test_gelu_fast_special_values():
    g, _ = gelu_fast(np.array([0.0, 1e-30, -1e-30, 50.0, -50.0, 1e6, -1e6, 3e38, -3e38]))
    assert g[0] == 0.0 and abs(g[1]) < 1e-29 and abs(g[2]) < 1e-29
    assert g[3] == np.float32(50.0) and abs(g[4]) < 1e-9
    # below -10 the result is z * 3.6e-12 (the CDF's fit held at its value at -10), not 0
    assert g[5] == np.float32(1e6) and abs(g[6]) <= 3.6e-6
    assert g[7] == np.float32(3e38) and np.isfinite(g[8])
    # GELU(z) - GELU(-z) = z holds to the fit's accuracy (sigma(g) + sigma(-g) = 1 exactly)
    z = np.linspace(-6.0, 6.0, 10001)
    a, _ = gelu_fast(z)
    b, _ = gelu_fast(-z)
    assert np.max(np.abs((a - b) - z.astype(np.float32))) <= 1e-5
