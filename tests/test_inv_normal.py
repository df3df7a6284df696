"""The single-precision inverse normal CDF of the Sobol path: its generated
coefficients, evaluated on the CPU in binary32 exactly as the kernel forms the
normal from a 30-bit coordinate, against scipy's ndtri (the library routine
the definition reduces to).  The kernel's formula: 2u = (2 xs + 1) 2^-30,
x = 1 - 2u, w = -ln(2u (2 - 2u)), z = -x Q(w), Q a polynomial in w - 4 for
w <= 8, else in sqrt(w) - 3.6."""
import os
import re

import numpy as np
from scipy.special import ndtri

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2309_10477_amd", "csrc", "inv_normal_coef.hpp")


def coefficients():
    text = open(HDR).read()
    arrays = {}
    for name, body in re.findall(r"constexpr float (\w+)\[\d+\] = \{([^}]*)\};", text):
        arrays[name] = np.array([np.float32(v.strip().rstrip("f")) for v in body.split(",")],
                                np.float32)
    scal = {n: np.float32(v) for n, v in re.findall(r"constexpr float (\w+) = ([0-9.]+)f;", text)}
    return arrays, scal


def horner(coef, t):
    p = np.full(t.shape, coef[0], np.float32)
    for c in coef[1:]:
        p = np.float32(p.astype(np.float64) * t + np.float64(c))  # one rounding (fma)
    return p


def inv_normal_bits(xs):
    arr, sc = coefficients()
    a = np.float32((2 * xs.astype(np.uint64) + 1).astype(np.float32) * np.float32(2.0 ** -30))
    x = np.float32(1.0) - a
    lg = np.log2((a * (np.float32(2.0) - a)).astype(np.float32)).astype(np.float32)
    ln2 = np.float32(np.log(2.0))
    w = np.float32(lg * -ln2)
    q = horner(arr["INV_NORMAL_CENTRAL"], np.float32(w - sc["INV_NORMAL_CENTER"]))
    tail = lg < -sc["INV_NORMAL_W_SPLIT"] / ln2
    qt = horner(arr["INV_NORMAL_TAIL"], np.float32(np.sqrt(w) - sc["INV_NORMAL_TAIL_CENTER"]))
    return np.float32(-x * np.where(tail, qt, q)), tail


def test_inverse_normal_against_ndtri():
    g = np.random.default_rng(1)
    xs = np.concatenate([np.arange(0, 4096, dtype=np.uint32),           # deep tail, u ~ 2^-31
                         (1 << 29) - 1 - np.arange(0, 4096, dtype=np.uint32),  # near u = 1/2
                         g.integers(0, 1 << 29, 400_000, dtype=np.uint32)])
    z, tail = inv_normal_bits(xs)
    u = (xs.astype(np.float64) + 0.5) * 2.0 ** -30
    ref = ndtri(u)
    # binary32 input rounding of 2u (relative 2^-24) moves z by at most
    # 2^-24 u / phi(z); the approximation adds 2.1e-7 relative, the
    # arithmetic a few roundings
    from scipy.stats import norm
    bound = 4e-7 * np.abs(ref) + 2.0 ** -24 * u / norm.pdf(ref) + 1e-7
    err = np.abs(z - ref)
    assert (err <= bound).all(), (float((err / bound).max()), int(np.argmax(err / bound)))
    assert tail.any() and not tail.all()
    assert (z <= 0).all()
