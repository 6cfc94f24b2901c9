"""Pins of the oracle's special functions: Legendre, real Y_lm, Lbar, wedges.

Each pin is something the paper or mathematics fixes independently of the oracle's code.
"""
import math

import numpy as np
import pytest
from scipy.special import eval_legendre, factorial2

from oracle.legendre import legendre, legendre_coefficients, lbar, legendre_integral
from oracle.ylm import real_ylm
from oracle.wedges import lbar_matrix, wedges


@pytest.mark.parametrize("ell", range(0, 17))
def test_legendre_matches_library_and_special_values(ell):
    x = np.linspace(-1, 1, 257)
    assert np.max(np.abs(legendre(ell, x) - eval_legendre(ell, x))) < 1e-14
    assert abs(float(legendre(ell, 1.0)) - 1.0) < 1e-14
    if ell % 2 == 0:
        # L_l(0) = (-1)^(l/2) (l-1)!! / l!!
        ref = (-1) ** (ell // 2) * (factorial2(ell - 1) if ell > 0 else 1.0) / (factorial2(ell) if ell > 0 else 1.0)
        assert abs(float(legendre(ell, 0.0)) - ref) < 1e-14
    # power-series coefficients against exact rationals (sympy)
    import sympy
    t = sympy.Symbol("t")
    exact = sympy.Poly(sympy.legendre(ell, t), t).all_coeffs()[::-1]
    c = legendre_coefficients(ell)
    for j, q in enumerate(exact):
        assert abs(c[j] - float(q)) <= 1e-15 * max(1.0, abs(float(q)))


def _rand_dirs(n, seed):
    v = np.random.default_rng(seed).normal(size=(n, 3))
    return v


@pytest.mark.parametrize("ell", [0, 1, 2, 3, 4, 6, 8, 12, 16])
def test_addition_theorem(ell):
    """eq. add-theorem: L_l(a.b) = 4 pi/(2l+1) sum_m Y_lm(a) Y_lm(b) (real harmonics)."""
    a = _rand_dirs(200, 1)
    b = _rand_dirs(200, 2)
    ah = a / np.linalg.norm(a, axis=1)[:, None]
    bh = b / np.linalg.norm(b, axis=1)[:, None]
    s = sum(real_ylm(ell, m, a) * real_ylm(ell, m, b) for m in range(-ell, ell + 1))
    ref = eval_legendre(ell, np.sum(ah * bh, axis=1))
    assert np.max(np.abs(4 * math.pi / (2 * ell + 1) * s - ref)) < 1e-13


def test_ylm_orthonormal_by_exact_quadrature():
    """Gauss-Legendre in cos(theta) x uniform phi grid is exact for these band-limited
    products, so <Y_lm, Y_l'm'> must be the identity."""
    lmax = 8
    xg, wg = np.polynomial.legendre.leggauss(lmax + 2)
    nphi = 2 * lmax + 3
    phi = 2 * math.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    v = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=-1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :]).ravel()
    lm = [(l, m) for l in range(lmax + 1) for m in range(-l, l + 1)]
    Y = np.stack([real_ylm(l, m, v) for l, m in lm])
    G = (Y * w) @ Y.T
    assert np.max(np.abs(G - np.eye(len(lm)))) < 1e-13


def test_ylm_low_order_closed_forms():
    """Textbook real harmonics: pins the m>0 cos / m<0 sin assignment and the absence of
    the Condon-Shortley phase in eq. real-Ylm."""
    v = _rand_dirs(50, 3)
    x, y, z = (v / np.linalg.norm(v, axis=1)[:, None]).T
    c1 = math.sqrt(3 / (4 * math.pi))
    assert np.allclose(real_ylm(1, 1, v), c1 * x, atol=1e-15, rtol=0)
    assert np.allclose(real_ylm(1, -1, v), c1 * y, atol=1e-15, rtol=0)
    assert np.allclose(real_ylm(1, 0, v), c1 * z, atol=1e-15, rtol=0)
    assert np.allclose(real_ylm(2, 0, v), math.sqrt(5 / (16 * math.pi)) * (3 * z * z - 1), atol=1e-15, rtol=0)
    assert np.allclose(real_ylm(2, 2, v), math.sqrt(15 / (16 * math.pi)) * (x * x - y * y), atol=1e-15, rtol=0)
    assert np.allclose(real_ylm(2, -2, v), math.sqrt(15 / (4 * math.pi)) * x * y, atol=1e-15, rtol=0)
    assert np.allclose(real_ylm(2, 1, v), math.sqrt(15 / (4 * math.pi)) * x * z, atol=1e-15, rtol=0)


@pytest.mark.parametrize("ell", [0, 2, 4, 8, 16])
def test_ylm_on_z_axis(ell):
    zhat = np.array([[0.0, 0.0, 2.5]])
    for m in range(-ell, ell + 1):
        ref = math.sqrt((2 * ell + 1) / (4 * math.pi)) if m == 0 else 0.0
        assert abs(float(real_ylm(ell, m, zhat)[0]) - ref) < 1e-13


@pytest.mark.parametrize("ell", [0, 1, 2, 4, 7, 16])
def test_lbar_against_quadrature(ell):
    a, b = 0.13, 0.71
    xg, wg = np.polynomial.legendre.leggauss(40)
    mu = 0.5 * (b - a) * xg + 0.5 * (b + a)
    ref = 0.5 * np.sum(wg * eval_legendre(ell, mu))
    assert abs(float(lbar(ell, a, b)) - ref) < 1e-15
    assert abs(float(legendre_integral(ell, a, b)) - ref * (b - a)) < 1e-15


def test_lbar_sum_rule():
    """sum_m dmu_m Lbar_l(m) = int_0^1 L_l = delta_l0 for even l (edges spanning [0, 1])."""
    edges = np.array([0.0, 0.05, 0.2, 0.37, 0.6, 0.81, 0.93, 1.0])
    for ell in range(0, 17, 2):
        s = np.sum(np.diff(edges) * lbar(ell, edges[:-1], edges[1:]))
        assert abs(s - (1.0 if ell == 0 else 0.0)) < 1e-14
    assert np.all(np.abs(lbar(0, edges[:-1], edges[1:]) - 1.0) < 1e-15)


@pytest.mark.parametrize("beta", [0.35, 0.75])
def test_kaiser_wedges_exact(beta):
    """Kaiser (eq. kaiser): (1 + beta mu^2)^2 has multipoles 1 + 2b/3 + b^2/5, 4b/3 + 4b^2/7,
    8b^2/35 and nothing above l = 4, so eq. wedge-est with lmax = 4 must return the exact
    mu-average of (1 + beta mu^2)^2 over any wedge."""
    poles = np.array([[1 + 2 * beta / 3 + beta ** 2 / 5], [4 * beta / 3 + 4 * beta ** 2 / 7], [8 * beta ** 2 / 35]])
    edges = np.array([0.0, 0.1, 0.33, 0.5, 0.9, 1.0])
    got = wedges(poles, [0, 2, 4], edges)[0]

    def prim(m):  # antiderivative of (1 + b m^2)^2
        return m + 2 * beta * m ** 3 / 3 + beta ** 2 * m ** 5 / 5
    ref = (prim(edges[1:]) - prim(edges[:-1])) / np.diff(edges)
    assert np.max(np.abs(got - ref)) < 1e-14
    # and extra zero multipoles change nothing
    poles16 = np.vstack([poles, np.zeros((6, 1))])
    got16 = wedges(poles16, list(range(0, 17, 2)), edges)[0]
    assert np.max(np.abs(got16 - ref)) < 1e-14
    assert lbar_matrix([0, 2, 4], edges).shape == (5, 3)
