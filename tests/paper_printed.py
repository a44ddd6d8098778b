"""The paper's printed real-space WT factors T_1..T_4 (Sec. 2, the four
piecewise equations following Eq. tau_l), valid for a = c dt/dx <= 1/2.

These are transcribed from the paper so that the oracle's T (built from the
Fourier-space definition, Eq. tau_l) can be checked against an independent
source.  One reading: the outermost piece of T_4 prints its denominator as
48 dt_i; the normalised 48 dt~_i is meant (only that makes T_4 continuous and
of unit sum).
"""
import numpy as np


def T1(x, a):
    x = np.abs(np.asarray(x, dtype=np.float64))
    return np.select(
        [x <= 0.5 - a, x <= 0.5 + a],
        [np.ones_like(x), (1 + 2 * a - 2 * x) / (4 * a)],
        0.0,
    )


def T2(x, a):
    x = np.abs(np.asarray(x, dtype=np.float64))
    return np.select(
        [x <= a, x <= 1 - a, x <= 1 + a],
        [(2 * a - a * a - x * x) / (2 * a), 1 - x, (a + 1 - x) ** 2 / (4 * a)],
        0.0,
    )


def T3(x, a):
    x = np.abs(np.asarray(x, dtype=np.float64))
    p0 = (9 - 4 * a * a - 12 * x * x) / 12
    p1 = (-8 * a**3 - 36 * a * a * (1 - 2 * x) - 3 * (1 - 2 * x) ** 3
          + 6 * a * (15 - 12 * x - 4 * x * x)) / (96 * a)
    p2 = (4 * a * a + 3 * (3 - 2 * x) ** 2) / 24
    p3 = (3 + 2 * a - 2 * x) ** 3 / (96 * a)
    return np.select(
        [x <= 0.5 - a, x <= 0.5 + a, x <= 1.5 - a, x <= 1.5 + a], [p0, p1, p2, p3], 0.0
    )


def T4(x, a):
    x = np.abs(np.asarray(x, dtype=np.float64))
    p0 = (3 * x**4 + a * (16 - 24 * x * x) + 18 * a * a * x * x - 8 * a**3 + 3 * a**4) / (24 * a)
    p1 = (4 - 6 * x * x + 3 * x**3 - a * a * (2 - 3 * x)) / 6
    p2 = (-(1 - x) ** 4 + 2 * a * (6 - 6 * x + x**3) - 6 * a * a * (1 - x) ** 2
          + 2 * a**3 * x - a**4) / (12 * a)
    p3 = (2 - x) * ((2 - x) ** 2 + a * a) / 6
    p4 = (a + 2 - x) ** 4 / (48 * a)
    return np.select(
        [x <= a, x <= 1 - a, x <= 1 + a, x <= 2 - a, x <= 2 + a], [p0, p1, p2, p3, p4], 0.0
    )


PRINTED_T = {1: T1, 2: T2, 3: T3, 4: T4}
