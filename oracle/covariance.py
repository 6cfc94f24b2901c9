"""Gaussian covariance of multipoles and wedges under linear Kaiser distortions (Sec. 4.1),
FP64.  Test infrastructure only: nothing in the GPU package imports it.

* pole_covariance_kernel(ells, beta): K[l, l'] = (2l+1)(2l'+1) int_{-1}^{1} (dmu/2)
  L_l L_l' (1 + beta mu^2)^4 -- the mu part of eq. pole-cov for P(k, mu) = (1+beta mu^2)^2 P(k)
  without shot noise (eq. kaiser).
* kaiser_gamma(ell_max, mu_edges, beta): eq. gamma, gamma_mn = sum_{l,l'} Lbar_l(mu_m)
  Lbar_l'(mu_n) K[l, l'] over even l, l' <= ell_max (eq. wedge-cov with eq. Lbar).
* correlation(C): C_mn / sqrt(C_mm C_nn); condition_number(M): largest over smallest singular
  value (Sec. 4.1 writes the ratio the other way round; the usual one is used here).

The mu integrals are done by scipy's fixed Gauss-Legendre rule with enough points to be exact
for the polynomial integrand (degree 2 ell_max + 8).
"""
from __future__ import annotations

import numpy as np
from scipy.special import roots_legendre

from .legendre import legendre
from .wedges import lbar_matrix


def pole_covariance_kernel(ells, beta: float) -> np.ndarray:
    ells = list(ells)
    x, w = roots_legendre(max(ells) + 5)
    k4 = (1.0 + beta * x * x) ** 4
    L = np.stack([legendre(l, x) for l in ells])
    raw = (L * (0.5 * w * k4)) @ L.T
    f = np.array([2 * l + 1 for l in ells], dtype=np.float64)
    return raw * f[:, None] * f[None, :]


def kaiser_gamma(ell_max: int, mu_edges, beta: float) -> np.ndarray:
    ells = list(range(0, ell_max + 1, 2))
    lb = lbar_matrix(ells, mu_edges)            # (n_mu, n_l)
    return lb @ pole_covariance_kernel(ells, beta) @ lb.T


def correlation(c) -> np.ndarray:
    c = np.asarray(c, dtype=np.float64)
    d = np.sqrt(np.diag(c))
    return c / d[:, None] / d[None, :]


def condition_number(m) -> float:
    s = np.linalg.svd(np.asarray(m, dtype=np.float64), compute_uv=False)
    return float(s[0] / s[-1])
