"""The cubic-box transverse-systematic test of Sec. 3.2 on the GPU path, l <= 16.

A Poisson box whose density is modulated sinusoidally across the line of sight puts a spike at
k_c = j k_f on modes with mu = 0; an observer 1e9 Mpc/h below the box makes the local line of
sight z-hat everywhere.

* 64^3: multipoles and wedges against the oracle run live (both precision forms).
* 512^3 and 1024^3 (full size, no oracle value): in the one k bin of the six axis modes every
  multipole must take the plane-parallel form (2l+1)[a L_l(0) + b] (Sec. 2.1 eq. Pell-ours with
  x-hat = z-hat), the non-uniform wedges of Sec. 3.1 must leave the spike in the first wedge
  only, and uniform wedges must carry it as eq. response predicts.
"""
from __future__ import annotations

import numpy as np
import pytest

from tests.parity_util import assert_pole_parity, oracle_params
from tests.systematics_util import leakage_ratio_theory, spike_decomposition, spike_edges

pytestmark = pytest.mark.gpu

FAR = (0.0, 0.0, -1e9)


def _plan(n, L, prec, lmax, max_group=0):
    from paper_1704_02357_amd import Plan
    return Plan(n, L, observer=FAR, window=3, interlaced=True, compensated=True, precision=prec,
                ell_max_hint=lmax, max_group=max_group)


SPIKE64 = dict(n=64, L=1000.0, j=8, ngal=200_000, seed=64)


@pytest.fixture(scope="module")
def spike64(gpu):
    """The 64^3 case and its oracle multipoles (computed once for both precision forms)."""
    from oracle.estimator import default_k_edges, multipoles
    from synth import modulated_box
    c = SPIKE64
    cat = modulated_box(c["L"], c["ngal"], c["seed"], c["j"], 0.8)
    edges = np.sort(np.concatenate([default_k_edges(c["n"], c["L"], 0.02), spike_edges(c["j"], c["L"])]))
    print("[oracle] spike box 64^3 l<=16", flush=True)
    ref = multipoles(cat, None, oracle_params(c["n"], c["L"], FAR, 3, True, True), 16, edges, workers=8)
    return cat, edges, ref


@pytest.mark.parametrize("prec", [1, 0])
def test_spike_box_64_l16_live_oracle(spike64, prec):
    from oracle.wedges import wedges as oracle_wedges
    from paper_1704_02357_amd import nonuniform_mu_edges, wedges
    cat, edges, ref = spike64
    print(f"[case] spike box 64^3 l<=16 prec={prec}", flush=True)
    plan = _plan(SPIKE64["n"], SPIKE64["L"], prec, 16)
    plan.paint(cat, None)
    got = plan.compute_multipoles(16, edges)
    plan.close()
    assert_pole_parity(got, ref, prec, "spike box 64^3 l<=16")
    mu = nonuniform_mu_edges(16)
    wg = wedges(got["poles"], 16, mu)
    wo = oracle_wedges(ref["poles"], ref["ells"], mu)
    ok = np.isfinite(wo)
    # per k bin, against the larger of the bin's wedges and its raw monopole P_0 + S
    scale = np.maximum(np.abs(wo), np.abs(ref["poles"][0] + ref["shot_noise"])[:, None])
    err = np.max(np.abs(wg - wo)[ok] / scale[ok])
    print(f"[parity] spike box wedges scaled_err={err:.3e}", flush=True)
    assert err <= (1e-5 if prec == 0 else 1e-12)


@pytest.mark.parametrize("n,L,j,ngal,max_group", [(512, 2500.0, 32, 2_000_000, 0), (1024, 3000.0, 64, 2_000_000, 24)])
def test_spike_box_full_size_l16(gpu, n, L, j, ngal, max_group):
    from paper_1704_02357_amd import nonuniform_mu_edges, wedges
    from synth import modulated_box
    cat = modulated_box(L, ngal, n + j, j, 0.8)
    edges = spike_edges(j, L)
    ells = list(range(0, 17, 2))
    fits = {}
    for prec in (1, 0):
        print(f"[case] spike box {n}^3 l<=16 prec={prec}", flush=True)
        plan = _plan(n, L, prec, 16, max_group)
        plan.paint(cat, None)
        r = plan.compute_multipoles(16, edges)
        plan.close()
        assert r["n_modes"][0] == 6
        a, b, misfit = spike_decomposition(r["poles"][:, 0], r["shot_noise"], ells)
        fits[prec] = a
        nu = wedges(r["poles"], 16, nonuniform_mu_edges(16)).ravel()
        uni_edges = np.linspace(0.0, 1.0, 10)
        uni = wedges(r["poles"], 16, uni_edges).ravel()
        dev = np.max(np.abs(uni / uni[0] - leakage_ratio_theory(16, uni_edges)))
        print(f"[property] {n}^3 prec={prec} a={a:.6e} b={b:.3e} misfit={misfit:.2e} "
              f"nonuniform_leak={np.max(np.abs(nu[1:] / nu[0])):.2e} uniform_vs_response={dev:.2e}", flush=True)
        assert a > 100 * abs(b)
        assert misfit < (1e-4 if prec == 0 else 1e-9)
        assert np.max(np.abs(nu[1:] / nu[0])) < 1e-3
        assert dev < 1e-3
    assert abs(fits[0] - fits[1]) <= 1e-5 * abs(fits[1])
