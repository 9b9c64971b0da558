#!/usr/bin/env python3
"""Coefficients of the FP64 2^f polynomial used by the product kernels.

2^f on |f| <= 1/2 by a near-minimax polynomial of degree 10: the Chebyshev
interpolant fitted with mpmath.chebyfit at 50 digits, coefficients rounded to
double.  Prints the coefficients (highest degree first) and the largest
relative error of the rounded polynomial, evaluated exactly on a fine grid
(about 3.2e-16; FP64 Horner evaluation adds rounding of the same order).
"""
import mpmath as mp

DEG = 10


def main() -> None:
    mp.mp.dps = 50
    f = lambda x: mp.power(2, x)  # noqa: E731
    coeffs, _ = mp.chebyfit(f, [-0.5, 0.5], DEG + 1, error=True)
    cd = [float(c) for c in coeffs]
    worst = mp.mpf(0)
    for k in range(8001):
        x = mp.mpf(-0.5) + mp.mpf(k) / 8000
        p = mp.mpf(0)
        for c in cd:
            p = p * x + mp.mpf(c)
        worst = max(worst, abs(p / f(x) - 1))
    for c in cd:
        print(repr(c))
    print(f"max relative error {float(worst):.3e}")


if __name__ == "__main__":
    main()
