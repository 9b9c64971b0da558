"""Parity bars of the kernel products against the FP64 oracle.

One reading for every product test (single- and multi-RHS, square and cross):

* The reference is the oracle evaluated on the original FP64 points and on the
  vector the call receives: FP64 q for FP64 products, the FP32 q (as the test
  rounds it for the call) for FP32 and BF16 products.  Every rounding the
  library does itself (offsets to FP32 or BF16, q to BF16, the exponent
  arithmetic) counts against the product.
* Bars: FP64 1e-12, FP32 1e-5, BF16-input 1e-2, both norm-wise
  (||y - y*|| / ||y*||) and element-wise (max_i |y_i - y*_i| / max_i |y*_i|).
* Where BF16's own rounding of q moves the exact product by more than its bar
  (smooth kernels on dense point sets: many comparable terms of both signs),
  the bar is 1.25 times that format floor, which the test computes with the
  oracle alone: the oracle on the BF16-rounded q against the oracle on q.  A
  test passes a floor only where it states why; the Gaussian products in the
  tests meet 1e-2 without one.
"""
import numpy as np
import torch

BAR = {"fp64": 1e-12, "fp32": 1e-5, "bf16": 1e-2}
DT = {"fp64": torch.float64, "fp32": torch.float32, "bf16": torch.float32}


def relerr(y, w) -> float:
    return float(np.linalg.norm(y - w) / max(np.linalg.norm(w), 1e-300))


def elemerr(y, w) -> float:
    return float(np.abs(y - w).max() / max(np.abs(w).max(), 1e-300))


def call_vector(q, prec):
    """The vector a product call of this precision receives (FP64 or FP32 values)."""
    q = np.asarray(q, dtype=np.float64)
    if prec == "fp64":
        return q
    return torch.from_numpy(np.ascontiguousarray(q)).float().double().numpy()


def bf16_round(q):
    """q rounded to bfloat16 (round to nearest even, by torch), as float64."""
    return torch.from_numpy(np.ascontiguousarray(q, dtype=np.float64)).float().to(torch.bfloat16).double().numpy()


def format_floor(ref, q32):
    """(norm-wise, element-wise) distance between the oracle product `ref` on
    the BF16-rounded q and on q itself: what BF16 inputs lose before any
    arithmetic."""
    a, b = ref(bf16_round(q32)), ref(q32)
    return relerr(a, b), elemerr(a, b)


def check(y, want, prec, floor=(0.0, 0.0), what=""):
    """Assert the product y against the reference at the precision's bar (or
    1.25 times a stated format floor, whichever is larger)."""
    n_bar = max(BAR[prec], 1.25 * floor[0])
    e_bar = max(BAR[prec], 1.25 * floor[1])
    rn, re = relerr(y, want), elemerr(y, want)
    assert rn <= n_bar and re <= e_bar, (what, prec, rn, n_bar, re, e_bar)
    return rn, re
