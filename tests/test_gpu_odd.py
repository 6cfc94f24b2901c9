"""GPU parity of pkm_compute_multipoles_all (every l <= l_max, odd ones as R_l = Im P_l of
eq. Pell-ours) against the FP64 oracle's all_multipoles, in both precision forms, with TSC,
interlacing and compensation, several l_max and field-group sizes; its even rows against
pkm_compute_multipoles on the same painted plan."""
from __future__ import annotations

import math

import numpy as np
import pytest

from tests.parity_util import TOL, assert_pole_parity, oracle_params, small_catalogs

pytestmark = pytest.mark.gpu

L = 300.0
OBS = (40.0, -25.0, -650.0)


def _edges(n):
    return np.arange(0.0, math.pi * n / L, 0.03)


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("n,lmax,max_group", [(32, 16, 0), (48, 15, 40), (32, 1, 0), (64, 7, 9)])
def test_all_ell_matches_oracle(gpu, prec, n, lmax, max_group):
    from oracle.estimator import all_multipoles
    from paper_1704_02357_amd import Plan
    d, r = small_catalogs(3000, 20000, L, seed=900 + n + lmax)
    print(f"[case] all l n={n} lmax={lmax} max_group={max_group} prec={prec}", flush=True)
    plan = Plan(n, L, observer=OBS, window=3, interlaced=True, compensated=True, precision=prec,
                ell_max_hint=16, max_group=max_group)
    plan.paint(d, r)
    got = plan.compute_multipoles_all(lmax, _edges(n))
    ref = all_multipoles(d, r, oracle_params(n, L, OBS, 3, True, True), lmax, _edges(n))
    assert got["n_transforms"] == (lmax + 1) ** 2 - 1 + 3 == ref["n_transforms"]
    assert got["poles"].shape == (lmax + 1, len(_edges(n)) - 1)
    assert_pole_parity(got, ref, prec, f"all l n={n} lmax={lmax}")
    # the odd rows carry a signal well above the tolerance (the comparison is not vacuous)
    if lmax >= 1:
        raw0 = np.abs(ref["poles"][0] + ref["shot_noise"])
        assert np.nanmax(np.abs(ref["poles"][1::2]) / raw0) > 100 * TOL[0]
    # even rows agree with the even-only call on the same painted plan
    if lmax >= 2:
        even = plan.compute_multipoles(lmax - lmax % 2, _edges(n))
        scale = np.maximum(np.abs(even["poles"]), np.abs(even["poles"][0] + even["shot_noise"])[None, :])
        ok = np.isfinite(even["poles"])
        err = np.max(np.abs(got["poles"][0::2][: even["poles"].shape[0]] - even["poles"])[ok] / scale[ok])
        assert err <= (1e-12 if prec else 2e-6), err
    plan.close()


def test_all_ell_rejects_bad_requests(gpu):
    from paper_1704_02357_amd import Plan, PkmError
    plan = Plan(16, L, observer=OBS, precision=1)
    with pytest.raises(PkmError) as e:          # nothing painted
        plan.compute_multipoles_all(3, _edges(16))
    assert e.value.status == 2
    d, r = small_catalogs(500, 3000, L, seed=3)
    plan.paint(d, r)
    for bad in (17, -1):
        with pytest.raises(PkmError) as e:
            plan.compute_multipoles_all(bad, _edges(16))
        assert e.value.status == 1
    with pytest.raises(PkmError):               # the even-only call keeps refusing odd l_max
        plan.compute_multipoles(3, _edges(16))
    plan.close()
