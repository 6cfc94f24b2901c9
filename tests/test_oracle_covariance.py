"""Pins of the Kaiser wedge covariance (Sec. 4.1, eq. pole-cov / eq. wedge-cov / eq. gamma)."""
import numpy as np
import pytest

from oracle.covariance import condition_number, correlation, kaiser_gamma, pole_covariance_kernel
from oracle.legendre import legendre
from oracle.systematics import nonuniform_mu_edges
from oracle.wedges import lbar_matrix


def test_kernel_without_distortions_is_diagonal():
    """beta = 0: orthogonality of Legendre polynomials, int (dmu/2) L_l L_l' = delta/(2l+1)."""
    ells = list(range(0, 17, 2))
    k = pole_covariance_kernel(ells, 0.0)
    assert np.allclose(k, np.diag([2 * l + 1 for l in ells]), rtol=0, atol=1e-12)


def test_kernel_monopole_closed_form():
    """K[0, 0] = int_0^1 (1 + beta mu^2)^4 dmu expanded by the binomial theorem."""
    from math import comb
    beta = 0.35
    exact = sum(comb(4, j) * beta ** j / (2 * j + 1) for j in range(5))
    assert abs(pole_covariance_kernel([0], beta)[0, 0] - exact) < 1e-15


def test_gamma_without_distortions_tends_to_independent_wedges():
    """beta = 0, ell_max -> infinity: the even Legendre series is complete on [0, 1], so the
    reconstructed wedges become independent with variance 1/width (eq. full-wedge-cov)."""
    edges = np.linspace(0.0, 1.0, 5)
    g = kaiser_gamma(400, edges, 0.0)
    target = np.diag(1.0 / np.diff(edges))
    assert np.max(np.abs(g - target)) < 0.02 * np.max(target)


@pytest.mark.parametrize("lmax,edges", [(4, np.linspace(0, 1, 4)), (8, np.linspace(0, 1, 6)),
                                        (16, None)])
def test_gamma_matches_monte_carlo_gaussian_modes(lmax, edges):
    """Simulate the estimator on one k shell: modes at mu on a fine grid, each with an
    exponentially distributed power of mean (1 + beta mu^2)^2 (a Gaussian complex amplitude),
    P_l = (2l+1)/N sum L_l(mu_i) |d_i|^2, wedges from eq. wedge-est.  N times the covariance
    over realisations must reproduce gamma (eq. trunc-Cmn with 2/N_k -> 1/N for independent
    modes)."""
    beta = 0.35
    edges = nonuniform_mu_edges(lmax) if edges is None else edges
    rng = np.random.default_rng(lmax)
    n_modes, reps = 400, 40000
    mu = (np.arange(n_modes) + 0.5) / n_modes
    ells = list(range(0, lmax + 1, 2))
    L = np.stack([legendre(l, mu) for l in ells])                      # (n_l, N)
    p = (1.0 + beta * mu * mu) ** 2
    pw = rng.exponential(1.0, size=(reps, n_modes)) * p[None, :]
    poles = (pw @ L.T) * (np.array([2 * l + 1 for l in ells]) / n_modes)[None, :]   # (reps, n_l)
    w = poles @ lbar_matrix(ells, edges).T                             # (reps, n_mu)
    cov = np.cov(w, rowvar=False) * n_modes
    g = kaiser_gamma(lmax, edges, beta)
    # mode grid of 400 points instead of the mu integral, and 4e4 realisations: a few percent
    err = np.max(np.abs(cov - g)) / np.max(np.abs(np.diag(g)))
    assert err < 0.04, err
    assert np.max(np.abs(correlation(cov) - correlation(g))) < 0.04


def test_condition_numbers_follow_sec_4_1():
    """Fig. condition: with N_mu = ell_max/2 + 1 wedges, uniform bins make gamma and Lbar
    ill-conditioned at large ell_max while the non-uniform bins of Sec. 3.1 stay moderate."""
    beta = 0.35
    out = {}
    for lmax in (4, 16):
        ells = list(range(0, lmax + 1, 2))
        uni = np.linspace(0, 1, lmax // 2 + 2)
        non = nonuniform_mu_edges(lmax)
        out[lmax] = [condition_number(kaiser_gamma(lmax, e, beta)) for e in (uni, non)] + \
                    [condition_number(lbar_matrix(ells, e)) for e in (uni, non)]
    g_uni4, g_non4, l_uni4, l_non4 = out[4]
    g_uni16, g_non16, l_uni16, l_non16 = out[16]
    assert g_uni4 < 1e3 and g_non4 < 1e3
    assert g_uni16 > 100 * g_non16 and l_uni16 > 10 * l_non16
    assert g_uni16 > 10 * g_uni4
