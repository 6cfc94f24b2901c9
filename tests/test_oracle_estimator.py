"""Pins of the oracle estimator O3 against independent tiers and closed forms."""
import math
from fractions import Fraction

import numpy as np
import pytest

from synth import Catalog, uniform_box
from oracle.cartesian import cartesian_fft_count, cartesian_multipoles, cartesian_terms, harmonic_fft_count
from oracle.direct import brute_force_multipoles, yamamoto_direct
from oracle.estimator import default_params, k_thresholds, mode_bins, multipoles
from oracle.global_los import global_multipoles, pkmu
from oracle.legendre import legendre
from oracle.mesh import int_freq

import os
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cat(n, seed, N, L, on_node=False, weights=True):
    r = np.random.default_rng(seed)
    if on_node:
        pos = -L / 2 + r.integers(0, N, (n, 3)) * (L / N)
    else:
        pos = -L / 2 + r.random((n, 3)) * L
    w = r.uniform(0.5, 1.5, n) if weights else np.ones(n)
    return Catalog(pos, w, np.full(n, n / L ** 3))


N, L = 8, 100.0
EDGES = np.arange(0.05, 0.3, 0.05)
OBS = (10.0, -20.0, -300.0)


@pytest.mark.parametrize("window,interlaced,compensated", [(3, True, True), (2, False, True), (1, False, False), (2, True, False)])
def test_o3_equals_o1_brute_force(window, interlaced, compensated):
    """Harmonic factorisation (eq. Fell) == literal Legendre-weighted DFT, l <= 16."""
    d, r = _cat(40, 1, N, L), _cat(300, 2, N, L)
    p = default_params(N, L, observer=OBS, window=window, interlaced=interlaced, compensated=compensated)
    ells = [0, 2, 4, 8, 16]
    o3 = multipoles(d, r, p, 16, EDGES, ells=ells)
    o1, cnt = brute_force_multipoles(d, r, p, ells, EDGES)
    scale = np.max(np.abs(o1), axis=1, keepdims=True)
    assert np.max(np.abs(o3["poles"] - o1) / scale) < 1e-12
    assert np.array_equal(o3["n_modes"], cnt.astype(np.int64))


@pytest.mark.parametrize("window", [1, 2])
def test_o3_equals_o2_yamamoto_on_nodes(window):
    """Particles on nodes, NGP/CIC, no interlacing/compensation: the mesh sums are exactly the
    galaxy-direct Yamamoto sums (eq. Pell-yama) on the same modes."""
    d, r = _cat(40, 3, N, L, on_node=True), _cat(300, 4, N, L, on_node=True)
    p = default_params(N, L, observer=OBS, window=window, interlaced=False, compensated=False)
    o3 = multipoles(d, r, p, 6, EDGES)
    o2, cnt = yamamoto_direct(d, r, p, [0, 2, 4, 6], EDGES)
    scale = np.max(np.abs(o2), axis=1, keepdims=True)
    assert np.max(np.abs(o3["poles"] - o2) / scale) < 1e-12


def test_o3_equals_o4_cartesian():
    d, r = _cat(40, 5, N, L), _cat(300, 6, N, L)
    p = default_params(N, L, observer=OBS, window=3, interlaced=True, compensated=True)
    ells = [0, 2, 4, 6, 8]
    o3 = multipoles(d, r, p, 8, EDGES)
    o4, _, nfft = cartesian_multipoles(d, r, p, ells, EDGES)
    scale = np.max(np.abs(o4), axis=1, keepdims=True)
    assert np.max(np.abs(o3["poles"] - o4) / scale) < 1e-11
    assert nfft == sum((l + 1) * (l + 2) // 2 for l in ells if l > 0)


def test_cartesian_expansion_reproduces_legendre():
    rng = np.random.default_rng(9)
    a = rng.normal(size=(30, 3)); a /= np.linalg.norm(a, axis=1)[:, None]
    b = rng.normal(size=(30, 3)); b /= np.linalg.norm(b, axis=1)[:, None]
    for ell in [2, 4, 6]:
        terms = cartesian_terms(ell)
        assert len(terms) == (ell + 1) * (ell + 2) // 2
        v = np.zeros(30)
        for xe, kt in terms.items():
            g = sum(c * np.prod(b ** np.array(ke), axis=1) for ke, c in kt.items())
            v += np.prod(a ** np.array(xe), axis=1) * g
        assert np.max(np.abs(v - legendre(ell, np.sum(a * b, axis=1)))) < 1e-12


def test_paper_fft_counts():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_fft_counts.txt")) if l.strip() and not l.startswith("#")]
    for row in rows:
        ell, mode, ours, cart = int(row[0]), row[1], int(row[2]), int(row[3])
        if mode == "all":
            assert harmonic_fft_count(ell) == ours and cartesian_fft_count(ell) == cart
        else:
            assert 2 * ell + 1 == ours and (ell + 1) * (ell + 2) // 2 == cart
    assert abs(1 - 9 / 15 - 0.40) < 1e-12
    assert round(525 / 153, 1) == 3.4


@pytest.mark.parametrize("interlaced,compensated,expect", [(True, True, 17), (False, True, 16), (False, False, 15), (True, False, 17)])
def test_transform_count(interlaced, compensated, expect):
    d, r = _cat(10, 7, N, L), _cat(50, 8, N, L)
    p = default_params(N, L, observer=OBS, window=2, interlaced=interlaced, compensated=compensated)
    assert multipoles(d, r, p, 4, EDGES)["n_transforms"] == expect


def test_k_thresholds_and_counts_exact():
    """Bin membership by integer thresholds equals exact rational comparison of k = 2 pi |n| / L."""
    n, Lb = 16, 20 * math.pi          # k = |n| / 10
    edges = [0.0, 0.1, 0.15, 0.3, 0.45, 0.8]
    thr = k_thresholds(edges, Lb)
    assert list(thr) == [0, 1, 3, 9, 21, 64]
    bins = mode_bins(n, thr)
    f = int_freq(n)
    cnt = np.zeros(len(edges) - 1, dtype=np.int64)
    ksum = np.zeros(len(edges) - 1)
    fe = [Fraction(e).limit_denominator(1000) for e in edges]
    for a in f:
        for b in f:
            for c in f:
                if -n // 2 in (a, b, c) or (a, b, c) == (0, 0, 0):
                    continue
                n2 = int(a * a + b * b + c * c)
                for i in range(len(edges) - 1):
                    if (10 * fe[i]) ** 2 <= n2 < (10 * fe[i + 1]) ** 2:
                        cnt[i] += 1
                        ksum[i] += math.sqrt(n2) / 10
    got = np.bincount(bins[bins >= 0], minlength=len(edges) - 1)
    assert np.array_equal(got, cnt)
    d = _cat(20, 1, n, Lb)
    p = default_params(n, Lb, window=2, interlaced=False, compensated=False)
    res = multipoles(d, None, p, 0, edges)
    with np.errstate(invalid="ignore"):
        assert np.allclose(res["k_mean"], ksum / cnt, rtol=1e-14, atol=0, equal_nan=True)
    assert np.array_equal(res["n_modes"], cnt)


def test_global_los_limit():
    """Observer receding along -z: local multipoles -> (2l+1) <|C|^2 L_l(mu)>/I - delta S."""
    n, Lb = 16, 200.0
    d, r = _cat(300, 11, n, Lb), _cat(2000, 12, n, Lb)
    edges = np.arange(0.03, 0.25, 0.03)
    glob, _ = global_multipoles(d, r, default_params(n, Lb), [0, 2, 4], edges, (0.0, 0.0, 1.0))
    scale = np.max(np.abs(glob[0]))
    err = []
    for dist in (1e4, 1e6, 1e12):
        p = default_params(n, Lb, observer=(0.0, 0.0, -dist * Lb), window=3, interlaced=True, compensated=True)
        err.append(np.max(np.abs(multipoles(d, r, p, 4, edges)["poles"] - glob)) / scale)
    # the local line of sight deviates from +z by O(L/D): the difference falls as 1/D
    assert 50 < err[0] / err[1] < 200
    assert err[2] < 1e-9
    # an observer at a finite distance differs at O((L/D)^2): the test above is not vacuous
    near = default_params(n, Lb, observer=(0.0, 0.0, -2.0 * Lb), window=3, interlaced=True, compensated=True)
    assert np.max(np.abs(multipoles(d, r, near, 4, edges)["poles"][1:] - glob[1:])) / scale > 1e-4


def test_pkmu_consistent_with_global_multipoles():
    """P(k, mu) in fine mu bins integrates back to the global-LOS monopole (mode-weighted)."""
    n, Lb = 16, 200.0
    d = _cat(500, 13, n, Lb)
    edges = np.arange(0.03, 0.25, 0.03)
    mue = np.linspace(0, 1, 6)
    p = default_params(n, Lb, window=2, interlaced=False, compensated=True)
    pk, cnt = pkmu(d, None, p, edges, mue, (0.0, 0.0, 1.0))
    g, gc = global_multipoles(d, None, p, [0], edges, (0.0, 0.0, 1.0))
    assert np.array_equal(cnt.sum(axis=1), gc.astype(np.int64))
    mono = np.nansum(pk * cnt, axis=1) / cnt.sum(axis=1)
    assert np.max(np.abs(mono - g[0])) / np.max(np.abs(g[0])) < 1e-12


def test_shot_noise_poisson_level():
    """Unclustered Poisson box, periodic mode, CIC with Jing's alias-sum compensation:
    S = 1/nbar exactly and the mode-weighted mean of P_0 (shot noise removed) is 0 within
    3 sigma, sigma = (1/nbar) sqrt(2 / N_modes) (Sec. 2.1 shot-noise term)."""
    n, Lb = 32, 500.0
    npart = 20000
    d = uniform_box(Lb, npart, seed=21)
    p = default_params(n, Lb, window=2, interlaced=False, compensated=True)
    edges = np.linspace(2 * math.pi / Lb * 0.999, math.pi * n / Lb, 12)
    res = multipoles(d, None, p, 0, edges)
    nbar = npart / Lb ** 3
    assert abs(res["shot_noise"] * nbar - 1.0) < 1e-14
    nm = res["n_modes"].sum()
    mean = np.sum(res["poles"][0] * res["n_modes"]) / nm
    assert abs(mean) < 3 * (1 / nbar) * math.sqrt(2.0 / nm)
