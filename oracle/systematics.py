"""Transverse-systematic toy model (Sec. 3.1), FP64.

* delta_l = (2l+1)/2 L_l(0): Legendre coefficients of a Dirac delta at mu = 0 (eq. delta-ell).
* christoffel(lmax, x, y): sum_{l<=lmax} (2l+1) L_l(x) L_l(y) summed term by term.
* response(lmax, mu) = -(lmax+1)/(2 mu) L_lmax(0) L_{lmax+1}(mu) (eq. response), and the same
  leakage obtained directly as -sum_{even l <= lmax} delta_l L_l(mu).
* nonuniform_mu_edges(lmax): edges 0 = mu_0 < mu_1 < ... < mu_{lmax/2+1} = 1 such that
  int_{mu_i}^{mu_{i+1}} L_{lmax+1}(mu)/mu dmu = 0 for i >= 1 (eq. nonuniform-bins), i.e. the
  roots in (0, 1) of G(mu) = G(1) with G(mu) = int_0^mu L_{lmax+1}(t)/t dt (a polynomial).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import polynomial as P

from .legendre import legendre, legendre_coefficients


def delta_ell(ell: int) -> float:
    return (2 * ell + 1) / 2.0 * float(legendre(ell, 0.0))


def christoffel(lmax: int, x, y):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return sum((2 * l + 1) * legendre(l, x) * legendre(l, y) for l in range(lmax + 1))


def response(lmax: int, mu):
    mu = np.asarray(mu, dtype=np.float64)
    return -(lmax + 1) / (2.0 * mu) * float(legendre(lmax, 0.0)) * legendre(lmax + 1, mu)


def leakage_direct(lmax: int, mu):
    """-sum over even l <= lmax of delta_l L_l(mu): what the truncated expansion of the
    delta function puts at mu (odd l have delta_l = 0)."""
    mu = np.asarray(mu, dtype=np.float64)
    return -sum(delta_ell(l) * legendre(l, mu) for l in range(0, lmax + 1, 2))


def _g_poly(lmax: int) -> np.ndarray:
    c = legendre_coefficients(lmax + 1)   # odd polynomial: c[0] = 0
    q = c[1:]                              # L_{lmax+1}(t)/t
    return P.polyint(q)


def nonuniform_mu_edges(lmax: int) -> np.ndarray:
    if lmax % 2 or lmax < 2:
        raise ValueError("lmax must be even and >= 2")
    g = _g_poly(lmax)
    h = g.copy()
    h[0] -= P.polyval(1.0, g)
    roots = P.polyroots(h)
    real = np.sort(np.real(roots[np.abs(np.imag(roots)) < 1e-9]))
    inner = real[(real > 1e-12) & (real < 1.0 - 1e-9)]
    if inner.size != lmax // 2:
        raise RuntimeError("unexpected number of edge roots")
    # polish each root by Newton steps on h with h' = L_{lmax+1}(mu)/mu
    dq = P.polyder(h)
    for _ in range(5):
        inner = inner - P.polyval(inner, h) / P.polyval(inner, dq)
    return np.concatenate([[0.0], inner, [1.0]])


def wedge_integral_of_leakage(lmax: int, a: float, b: float) -> float:
    """int_a^b L_{lmax+1}(mu)/mu dmu (zero for every non-first non-uniform bin)."""
    g = _g_poly(lmax)
    return float(P.polyval(b, g) - P.polyval(a, g))
