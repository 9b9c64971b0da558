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


TAB_HDR = os.path.join(os.path.dirname(__file__), "..", "paper_1408_1237_amd", "csrc", "exp2_table.h")


def _table_header(size: int = 256):
    src = open(TAB_HDR).read()
    deg = {256: 4, 4096: 2}[size]
    poly = src[src.index(f"EXP2_POLY{size}[{deg + 1}] = {{"):]
    poly = [float(v) for v in re.findall(r"[-0-9.e+]+", poly[poly.index("{") + 1: poly.index("}")])]
    tab = src[src.index(f"EXP2_TABLE{size}[{size}] = {{"):]
    tab = [float(v) for v in re.findall(r"[-0-9.e+]+", tab[tab.index("{") + 1: tab.index("}")])]
    return poly, tab


def test_exp2_table_correctly_rounded():
    # the FP64 product's table holds 2^(j/256) rounded to nearest double
    import mpmath as mp
    mp.mp.dps = 50
    poly, tab = _table_header()
    assert len(poly) == 5 and poly[-1] == 1.0 and len(tab) == 256
    for j, v in enumerate(tab):
        assert v == float(mp.power(2, mp.mpf(j) / 256))


def test_exp2_x256_scheme_float64():
    # 2^(x/256) = 2^((n - j)/256) 2^(j/256) p(x - n), n = rint(x), j = n mod 256,
    # evaluated in float64 as the kernel does (with separate multiply and add in
    # place of the fused operations), against mpmath over the argument range the
    # kernel feeds it, including the clamp value -2000 * 256 (result 0)
    import mpmath as mp
    mp.mp.dps = 40
    poly, tab = _table_header()
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.uniform(-1100 * 256, 256 * 256, 3000), rng.uniform(-512, 512, 1000),
                         np.arange(-300, 300) + 0.5, [0.0, -0.5, 0.5, 255.5, -256.5]])
    worst = 0.0
    for x in xs:
        n = np.rint(x)
        f = x - n
        i = int(n)
        p = poly[0]
        for c in poly[1:]:
            p = p * f + c
        got = np.ldexp(p * tab[i & 255], i >> 8)
        want = mp.power(2, mp.mpf(float(x)) / 256)
        if want < mp.mpf(2) ** -1000:
            continue
        worst = max(worst, float(abs(mp.mpf(float(got)) / want - 1)))
    assert worst < 5e-16
    i = -2000 * 256
    assert np.ldexp(1.0 * tab[i & 255], i >> 8) == 0.0


def test_exp2_table4096_correctly_rounded_and_poly():
    # the 4096-entry form of the products at d <= 3: 2^(j/4096) rounded to
    # nearest double, and the degree-2 polynomial of 2^(f/4096) on |f| <= 1/2
    # evaluated exactly against mpmath: 2.5e-14 relative, within a factor 1.2 of
    # the degree-2 minimax bound h^3 / 24 (h = ln 2 / 8192)
    import mpmath as mp
    mp.mp.dps = 50
    poly, tab = _table_header(4096)
    assert len(poly) == 3 and len(tab) == 4096
    for j in range(0, 4096, 11):
        assert tab[j] == float(mp.power(2, mp.mpf(j) / 4096))
    assert tab[4095] == float(mp.power(2, mp.mpf(4095) / 4096))
    worst = 0.0
    for k in range(2001):
        f = Fraction(-1, 2) + Fraction(k, 2000)
        p = Fraction(0)
        for v in poly:
            p = p * f + Fraction(v)
        ref = mp.power(2, mp.mpf(f.numerator) / f.denominator / 4096)
        worst = max(worst, float(abs(mp.mpf(p.numerator) / p.denominator / ref - 1)))
    h = np.log(2.0) / 8192
    assert 0.5 * h ** 3 / 24 < worst < 1.2 * h ** 3 / 24 and worst < 3e-14


def test_exp2_x4096_scheme_float64():
    # 2^(x/4096) = 2^((n - j)/4096) 2^(j/4096) p(x - n) in float64 against mpmath,
    # including the clamp value -2000 * 4096 (result 0)
    import mpmath as mp
    mp.mp.dps = 40
    poly, tab = _table_header(4096)
    rng = np.random.default_rng(5)
    xs = np.concatenate([rng.uniform(-1100 * 4096, 256 * 4096, 3000), rng.uniform(-8192, 8192, 1000),
                         np.arange(-300, 300) + 0.5, [0.0, -0.5, 0.5, 4095.5, -4096.5]])
    worst = 0.0
    for x in xs:
        n = np.rint(x)
        f = x - n
        i = int(n)
        p = poly[0]
        for c in poly[1:]:
            p = p * f + c
        got = np.ldexp(p * tab[i & 4095], i >> 12)
        want = mp.power(2, mp.mpf(float(x)) / 4096)
        if want < mp.mpf(2) ** -1000:
            continue
        worst = max(worst, float(abs(mp.mpf(float(got)) / want - 1)))
    assert worst < 3e-14
    i = -2000 * 4096
    assert np.ldexp(1.0 * tab[i & 4095], i >> 12) == 0.0
