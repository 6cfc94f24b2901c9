"""Pins of the transverse-systematic helpers (Sec. 3.1)."""
import os

import numpy as np
import pytest

from oracle.legendre import legendre
from oracle.systematics import (christoffel, delta_ell, leakage_direct, nonuniform_mu_edges,
                                response, wedge_integral_of_leakage)
from tests.systematics_util import leakage_ratio_theory, spike_decomposition, spike_edges

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


# ---------------------------------------------------------------------------------------------
# Cubic-box transverse systematic (Sec. 3.2) through the oracle estimator
# ---------------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def spike_oracle():
    from oracle.estimator import default_params, multipoles
    from synth import modulated_box
    n, L, j = 32, 1000.0, 4
    cat = modulated_box(L, 100_000, 11, j, 0.8)
    p = default_params(n, L, observer=(0.0, 0.0, -1e9))
    return multipoles(cat, None, p, 16, spike_edges(j, L), workers=8)


def test_spike_bin_is_plane_parallel(spike_oracle):
    """Far observer: the local-LOS multipoles of the spike bin reduce to the plane-parallel form
    (2l+1) sum_modes |C|^2 L_l(mu) up to l = 16 (Sec. 2.1 eq. Pell-ours with x-hat = z-hat)."""
    r = spike_oracle
    assert r["n_modes"][0] == 6
    a, b, misfit = spike_decomposition(r["poles"][:, 0], r["shot_noise"], r["ells"])
    assert a > 100 * abs(b) > 0 and misfit < 1e-10


def test_nonuniform_wedges_isolate_the_spike(spike_oracle):
    """Sec. 3.2: with the non-uniform mu edges of Sec. 3.1 the transverse spike stays in the first
    wedge (the rest carry only shot-noise residue, here < 1e-3 of it); with uniform edges every
    wedge is contaminated as the response of eq. response predicts."""
    from oracle.wedges import wedges
    r = spike_oracle
    nu = wedges(r["poles"], r["ells"], nonuniform_mu_edges(16)).ravel()
    assert np.max(np.abs(nu[1:] / nu[0])) < 1e-3
    uni_edges = np.linspace(0.0, 1.0, 10)
    uni = wedges(r["poles"], r["ells"], uni_edges).ravel()
    th = leakage_ratio_theory(16, uni_edges)
    assert np.max(np.abs(uni / uni[0] - th)) < 1e-3
    assert np.min(np.abs(th[1:])) > 0.02
