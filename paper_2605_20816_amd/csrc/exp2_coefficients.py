"""Coefficients of the FP64 2^f of pd_math.h: the Chebyshev interpolant of
degree 11 of 2^f on [-1/2, 1/2] (mpmath.chebyfit, 50 digits), highest degree
first, rounded to FP64; and the largest error of its FMA Horner evaluation over
sampled arguments, in units in the last place of the exact value.

    python exp2_coefficients.py
"""
import random

import mpmath as mp
import numpy as np


def coefficients():
    mp.mp.dps = 50
    poly, err = mp.chebyfit(lambda x: mp.power(2, x), [-0.5, 0.5], 12, error=True)
    return [float(v) for v in poly], err


def horner_fma(c, t):
    p = c[0]
    for k in c[1:]:
        p = float(mp.mpf(p) * mp.mpf(t) + mp.mpf(k))  # one rounding per step
    return p


if __name__ == "__main__":
    c, err = coefficients()
    print("interpolation error", mp.nstr(err, 5))
    for v in c:
        print(repr(v))
    rng = random.Random(1)
    worst = 0.0
    for t in [rng.uniform(-0.5, 0.5) for _ in range(20000)] + [-0.5, 0.5, 0.0]:
        ref = mp.power(2, mp.mpf(t))
        worst = max(worst, float(abs(mp.mpf(horner_fma(c, t)) - ref) / np.spacing(float(ref))))
    print("largest error (ulp)", worst)
