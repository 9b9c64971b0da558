"""The BF16 input format's own floor, computed with the oracle alone (CPU).

A BF16-input product rounds q to bfloat16 (8 significant bits) before any
arithmetic.  The oracle on the rounded q against the oracle on q measures what
that rounding alone costs; where it exceeds the 1e-2 bar the GPU tests hold
the product to 1.25 times it (tests/parity.py).  These tests pin where that
happens on the tests' own shapes: the Matern-3/2 kernel at d = 12 and 16 (flat
near zero distance: many comparable terms of both signs in every row), and not
the Gaussian shapes, which keep the plain 1e-2 bar.
"""
import numpy as np
import pytest

import oracle
from paper_1408_1237_amd import workloads
from parity import bf16_round, call_vector, format_floor


def test_bf16_rounding_is_round_to_nearest_even():
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even significand
    q = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(2.0 + 2.0 ** -7), 3.0e-3])
    r = bf16_round(q)
    assert r[0] == 1.0 and r[1] == 1.0 + 2 * 2.0 ** -7 and r[2] == -2.0
    assert abs(r[3] - q[3]) <= 2.0 ** -8 * abs(q[3])


@pytest.mark.parametrize("d", [12, 16])
def test_matern_bf16_floor_reaches_the_bar(d):
    # the shape of the Matern matrix-core vs VALU test (n = 1900, h = 0.8 sqrt(d))
    n = 1900
    x = workloads.random_points(120 + d, n, d, 1.0, kind="normal")
    q32 = call_vector(workloads.random_vector(121 + d, n), "bf16")
    h = 0.8 * np.sqrt(d)
    fn, fe = format_floor(lambda v: oracle.matern_mvp(x, h, v, shift=0.03), q32)
    assert fn > 1e-3
    if d == 16:
        assert fn > 1e-2  # the bar alone would fail on the format, not on the kernel


@pytest.mark.parametrize("d", [2, 8, 16, 64])
def test_gaussian_bf16_floor_is_below_the_bar(d):
    # the shape of the Gaussian dimension sweep (n = 700, sigma = 0.5 sqrt(d)):
    # q's rounding alone leaves at least half the 1e-2 bar to the kernel
    n = 700
    x = workloads.random_points(300 + d, n, d, 1.0, kind="normal")
    q32 = call_vector(workloads.random_vector(400 + d, n), "bf16")
    sigma = 0.5 * np.sqrt(d)
    fn, fe = format_floor(lambda v: oracle.mvp(x, sigma, v, shift=0.1), q32)
    assert fn < 5e-3 and fe < 5e-3
