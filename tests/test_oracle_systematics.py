"""Pins of the transverse-systematic helpers (Sec. 3.1)."""
import os

import numpy as np
import pytest

from oracle.legendre import legendre
from oracle.systematics import (christoffel, delta_ell, leakage_direct, nonuniform_mu_edges,
                                response, wedge_integral_of_leakage)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_delta_ell_hand_values():
    # (2l+1)/2 L_l(0): 1/2, 5/2 (-1/2), 9/2 (3/8), 13/2 (-5/16)
    assert [delta_ell(l) for l in (0, 2, 4, 6)] == [0.5, -1.25, 27 / 16, -65 / 32]
    assert all(delta_ell(l) == 0.0 for l in (1, 3, 5))


@pytest.mark.parametrize("lmax", [2, 4, 8, 16])
def test_christoffel_closed_form(lmax):
    rng = np.random.default_rng(lmax)
    x, y = rng.uniform(-1, 1, 50), rng.uniform(-1, 1, 50)
    closed = (lmax + 1) / (y - x) * (legendre(lmax, x) * legendre(lmax + 1, y) - legendre(lmax, y) * legendre(lmax + 1, x))
    assert np.max(np.abs(christoffel(lmax, x, y) - closed)) < 1e-10 * lmax ** 2


@pytest.mark.parametrize("lmax", [4, 8, 16])
def test_response_equals_truncated_delta(lmax):
    """eq. response (with L_lmax(0), the consistent form) equals minus the truncated Legendre
    series of the delta function, term by term."""
    mu = np.linspace(0.01, 1.0, 200)
    assert np.max(np.abs(response(lmax, mu) - leakage_direct(lmax, mu))) < 1e-11


def _golden_edges():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "nonuniform_mu_edges.txt")) if l.strip() and not l.startswith("#")]
    return [(int(r[0]), int(r[1]), float(r[2])) for r in rows]


@pytest.mark.parametrize("lmax,nbins,w_uniform", _golden_edges())
def test_nonuniform_edges(lmax, nbins, w_uniform):
    e = nonuniform_mu_edges(lmax)
    assert e.size == nbins + 1 and e[0] == 0.0 and e[-1] == 1.0
    assert np.all(np.diff(e) > 0)
    for i in range(1, nbins):
        assert abs(wedge_integral_of_leakage(lmax, e[i], e[i + 1])) < 1e-12
    assert abs(wedge_integral_of_leakage(lmax, e[0], e[1])) > 1e-3
    assert abs((e[1] - e[0]) - w_uniform) < 0.06
    # bins narrow towards mu = 1 after the first few (Sec. 3.1)
    assert np.diff(e)[-1] < np.diff(e)[1]
