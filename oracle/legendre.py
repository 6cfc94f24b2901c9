"""Legendre polynomials and wedge-averaged Legendre polynomials (FP64).

Sec. 2.2: eq. Ptrue expands P(k, mu) in L_l(mu); eq. Lbar defines the mean of L_l over a
mu wedge [mu_m, mu_{m+1}].
"""
from __future__ import annotations

import numpy as np


def legendre(ell: int, x):
    """L_ell(x) by the three-term (Bonnet) recurrence
    (n+1) L_{n+1} = (2n+1) x L_n - n L_{n-1}."""
    x = np.asarray(x, dtype=np.float64)
    if ell < 0:
        raise ValueError("ell must be >= 0")
    p0 = np.ones_like(x)
    if ell == 0:
        return p0
    p1 = x.copy()
    for n in range(1, ell):
        p0, p1 = p1, ((2 * n + 1) * x * p1 - n * p0) / (n + 1)
    return p1


def legendre_coefficients(ell: int) -> np.ndarray:
    """Power-series coefficients c_j with L_ell(x) = sum_j c_j x^j (j = 0..ell).

    Built from the same recurrence on coefficient vectors."""
    p0 = np.zeros(ell + 1)
    p0[0] = 1.0
    if ell == 0:
        return p0
    p1 = np.zeros(ell + 1)
    p1[1] = 1.0
    for n in range(1, ell):
        xp1 = np.roll(p1, 1)
        xp1[0] = 0.0
        p0, p1 = p1, ((2 * n + 1) * xp1 - n * p0) / (n + 1)
    return p1


def legendre_integral(ell: int, a, b):
    """Integral of L_ell over [a, b].

    Uses (2l+1) L_l = d/dx [L_{l+1} - L_{l-1}] for l >= 1 and b - a for l = 0."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if ell == 0:
        return b - a
    fb = legendre(ell + 1, b) - legendre(ell - 1, b)
    fa = legendre(ell + 1, a) - legendre(ell - 1, a)
    return (fb - fa) / (2 * ell + 1)


def lbar(ell: int, mu_lo, mu_hi):
    """Mean Legendre polynomial over a wedge (eq. Lbar): (1/(b-a)) int_a^b L_ell(mu) dmu."""
    mu_lo = np.asarray(mu_lo, dtype=np.float64)
    mu_hi = np.asarray(mu_hi, dtype=np.float64)
    return legendre_integral(ell, mu_lo, mu_hi) / (mu_hi - mu_lo)
