"""The FP64 2^f polynomial of the product kernels, checked on the host.

The coefficients are read from the kernel header and the polynomial is evaluated
exactly (rational arithmetic) against 2^f from mpmath at 60 digits on
|f| <= 1/2, and then in float64 Horner form against numpy's exp2.
"""
import os
import re
from fractions import Fraction

import numpy as np

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_1408_1237_amd", "csrc", "krr_internal.h")


def _coeffs():
    src = open(HDR).read()
    body = src[src.index("double exp2_f64(double a)"):]
    body = body[: body.index("return")]
    vals = re.findall(r"(?:double p = |__builtin_fma\(p, f, )([0-9.e+-]+)", body)
    return [float(v) for v in vals]


def test_exp2_poly_exact_error():
    import mpmath as mp
    mp.mp.dps = 60
    c = _coeffs()
    assert len(c) == 11 and c[-1] == 1.0
    worst = 0.0
    for k in range(2001):
        f = Fraction(-1, 2) + Fraction(k, 2000)
        p = Fraction(0)
        for v in c:
            p = p * f + Fraction(v)
        ref = mp.power(2, mp.mpf(f.numerator) / f.denominator)
        worst = max(worst, float(abs(mp.mpf(p.numerator) / p.denominator / ref - 1)))
    assert worst < 4e-16


def test_exp2_poly_float64_horner():
    c = _coeffs()
    f = np.linspace(-0.5, 0.5, 100001)
    p = np.full_like(f, c[0])
    for v in c[1:]:
        p = p * f + v
    rel = np.abs(p / np.exp2(f) - 1)
    assert rel.max() < 1e-15
