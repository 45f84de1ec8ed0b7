"""Random-pure-state logarithmic negativity, Sec. VII.A Eq. 6.

Oracle, test infrastructure only.

With R = 2 sqrt(d_A d_B / d_C):
    E = log2[ (2/pi) asin(1/R) + 2 (1 + 2 R^2) / (3 pi R) sqrt(1 - 1/R^2) ]   (R >= 1)
and E = 0 for R < 1 (zero negativity below half the system, Sec. VII.A).
The formula is the large-dimension limit; finite sizes deviate from it.
"""
from __future__ import annotations

import math


def random_state_logneg(d_a: int, d_b: int, d_c: int) -> float:
    r = 2.0 * math.sqrt(d_a * d_b / d_c)
    if r <= 1.0:
        return 0.0
    x = (2.0 / math.pi) * math.asin(1.0 / r) + 2.0 * (1.0 + 2.0 * r * r) / (3.0 * math.pi * r) * math.sqrt(
        1.0 - 1.0 / (r * r))
    return math.log2(x)
