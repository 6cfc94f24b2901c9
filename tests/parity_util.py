"""Shared helpers for the GPU parity tests: seeded inputs, both sides, the pass rule."""
from __future__ import annotations

import numpy as np

from synth import Catalog

# Tolerances of the two precision forms: relative error per k bin, measured against
# max(|P_l^oracle(k)|, P_0^raw(k)) with P_0^raw = P_0 + S, because high-l multipoles sit near
# zero while FP32 rounding scales with the raw power.
TOL = {0: 1e-5, 1: 1e-12}


def small_catalogs(n_data, n_rand, box_len, seed, weights=True, origin=None):
    rng = np.random.default_rng(seed)
    o = np.full(3, -0.5 * box_len) if origin is None else np.asarray(origin)
    pd = o + rng.random((n_data, 3)) * box_len
    pr = o + rng.random((n_rand, 3)) * box_len
    wd = rng.uniform(0.5, 1.5, n_data) if weights else np.ones(n_data)
    wr = rng.uniform(0.5, 1.5, n_rand) if weights else np.ones(n_rand)
    nb = n_data / box_len ** 3
    return Catalog(pd, wd, np.full(n_data, nb)), (Catalog(pr, wr, np.full(n_rand, nb)) if n_rand else None)


def oracle_params(nmesh, box_len, observer, window, interlaced, compensated):
    from oracle.estimator import default_params
    return default_params(nmesh, box_len, observer=observer, window=window, interlaced=interlaced,
                          compensated=compensated)


def pole_errors(gpu: dict, orc: dict):
    """Return (max scaled error, max plain relative error) over all l and bins."""
    pg, po = np.asarray(gpu["poles"]), np.asarray(orc["poles"])
    raw0 = po[0] + orc["shot_noise"]
    scale = np.maximum(np.abs(po), np.abs(raw0)[None, :])
    ok = np.isfinite(po)
    assert np.array_equal(ok, np.isfinite(pg)), "empty bins differ"
    scaled = np.max(np.abs(pg - po)[ok] / scale[ok]) if ok.any() else 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.abs(pg - po) / np.abs(po)
    plain = np.max(rel[ok & np.isfinite(rel)]) if ok.any() else 0.0
    return scaled, plain


def assert_pole_parity(gpu: dict, orc: dict, precision: int, label: str = ""):
    assert np.array_equal(np.asarray(gpu["n_modes"]), np.asarray(orc["n_modes"])), f"{label}: mode counts differ"
    km_ok = np.isfinite(orc["k_mean"])
    # k_mean is a sum of n_b positive FP64 terms on both sides, in different orders: the
    # recursive-summation bound (n_b - 1) u, u = 2^-53, with a floor of 1e-13
    cnt = np.asarray(orc["n_modes"], dtype=np.float64)[km_ok]
    km_tol = np.maximum(1e-13, cnt * 2.0 ** -53)
    km_err = np.abs(gpu["k_mean"][km_ok] - orc["k_mean"][km_ok]) / np.abs(orc["k_mean"][km_ok])
    assert np.all(km_err <= km_tol), f"{label}: k_mean rel err {km_err.max():.2e}"
    for key in ("alpha", "norm_I", "shot_noise"):
        assert abs(gpu[key] - orc[key]) <= 1e-13 * abs(orc[key]) + 1e-300, f"{label}: {key}"
    scaled, plain = pole_errors(gpu, orc)
    print(f"[parity] {label} scaled_err={scaled:.3e} plain_rel_err={plain:.3e} tol={TOL[precision]:.0e}", flush=True)
    assert scaled <= TOL[precision], f"{label}: scaled error {scaled:.3e} > {TOL[precision]:.0e}"
