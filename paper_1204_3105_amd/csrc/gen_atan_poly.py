"""Fit the odd polynomial used by the FP32 near field for atan(t), |t| <= 1.

atan(t) = t * Q(t^2) with Q a polynomial of degree n in x = t^2 on
[0, 1] (t = min(|x|, |y|) / max(|x|, |y|), no further reduction).  The
coefficients come from a weighted least-squares fit of atan(sqrt(x))/sqrt(x)
on Chebyshev nodes (near-minimax in relative error), refined by a few Lawson iterations on a dense grid.  Prints the C
initializer and the max relative error of the polynomial in float64 and in
float32 Horner evaluation.
"""
import math
import sys

import numpy as np


def fit(n):
    b = 1.0
    k = np.arange(6000)
    x = 0.5 * b * (1 - np.cos(math.pi * (k + 0.5) / len(k)))
    f = np.where(x > 0, np.arctan(np.sqrt(x)) / np.sqrt(np.maximum(x, 1e-300)), 1.0)
    V = np.vander(x, n + 1, increasing=True)
    w = np.ones_like(x)
    for _ in range(80):   # Lawson: reweight toward the largest errors
        c = np.linalg.lstsq(V * w[:, None], f * w, rcond=None)[0]
        e = np.abs(V @ c - f)
        w = w * (e / e.max() + 1e-3) ** 0.5
        w /= w.max()
    return c


def check(c):
    t = np.linspace(0, 1.0, 400001)
    ref = np.arctan(t)
    x = t * t
    p = np.zeros_like(t)
    for ci in reversed(c):
        p = p * x + ci
    e64 = np.max(np.abs(t * p - ref) / np.maximum(ref, 1e-30))
    t32 = t.astype(np.float32)
    x32 = (t32 * t32).astype(np.float32)
    p32 = np.zeros_like(t32)
    for ci in reversed(c):
        p32 = (p32 * x32 + np.float32(ci)).astype(np.float32)
    e32 = np.max(np.abs((t32 * p32).astype(np.float64) - np.arctan(t32.astype(np.float64))))
    return e64, e32


if __name__ == "__main__":
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 7
    c = fit(n)
    e64, e32 = check(c)
    print("// atan(t) = t * sum_k c_k t^(2k), |t| <= 1; max rel err %.2e (exact "
          "arithmetic), max abs err %.2e (float32 Horner)" % (e64, e32))
    print("static constexpr float kAtanPoly[%d] = {%s};" % (
        len(c), ", ".join("%.9ef" % v for v in c)))
