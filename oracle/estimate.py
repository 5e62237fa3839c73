"""Iteration estimate of the paper's section 1 -- TEST INFRASTRUCTURE.

The power iteration converges at the rate at which alpha^k goes to zero, so reaching a
tolerance tau takes about log10(tau) / log10(alpha) iterations (section 1, which quotes
85, 269, 48, 128 and 43 for five settings).
"""
import math


def iterations(tau: float, alpha: float) -> float:
    return math.log10(tau) / math.log10(alpha)


def rounded(tau: float, alpha: float) -> int:
    return int(math.floor(iterations(tau, alpha) + 0.5))
