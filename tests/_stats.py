"""Acceptance thresholds for Monte Carlo comparisons.

One entry is accepted within 3 combined standard errors (two-sided false
alarm 0.27 % for a normal estimate).  A comparison over k entries at once
uses the Bonferroni threshold that keeps the family-wise false alarm at the
same 0.27 %: z_k = Phi^-1(1 - 0.0027 / (2 k)); z_1 = 3.0.
"""
from scipy.stats import norm

FAMILY_ALPHA = 0.0026997960632601866  # 2 * (1 - Phi(3))


def z_crit(k=1):
    """Largest accepted |z| of each of k entries compared together."""
    k = max(1, int(k))
    return float(norm.isf(FAMILY_ALPHA / (2 * k)))


def z(a, b, sa, sb):
    import numpy as np
    den = np.sqrt(np.square(sa) + np.square(sb))
    return abs(a - b) / den
