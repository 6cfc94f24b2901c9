"""Pins of the oracle's mode-list evaluators, which the GPU parity tests use at mesh sizes
whose full grid does not fit in host memory:

* ``shell_modes`` lists exactly the modes the full-grid bin assignment puts in each bin;
* ``yamamoto_at_modes`` over those modes equals the FFT oracle (O3) exactly for particles on
  mesh nodes painted with NGP (no interlacing, no compensation): the mesh transform then is
  the galaxy sum at the same k (Sec. 2.1, eq. Pell-yama against eq. Pell-ours);
* ``combined_at_modes`` (direct sum over painted taps) equals the FFT-based combine for every
  window, with and without interlacing and compensation.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle.direct import combined_at_modes, shell_modes, yamamoto_at_modes
from oracle.estimator import default_params, density_fields, k_thresholds, mode_bins, multipoles
from oracle.mesh import int_freq
from synth import Catalog


@pytest.mark.parametrize("n", [16, 24])
def test_shell_modes_match_full_grid(n):
    thr = np.array([0, 1, 3, 4, 9, 20, 21, 50, 51, 52, 100, 101, 3 * (n // 2) ** 2 + 5])
    nb = thr.size - 1
    modes, b = shell_modes(n, thr, range(nb))
    mb = mode_bins(n, thr)
    f = int_freq(n)
    grid = np.stack(np.meshgrid(f, f, f, indexing="ij"), axis=-1)
    for i in range(nb):
        ref = np.sort(grid[mb == i].view([("", np.int64)] * 3).ravel())
        got = np.sort(np.ascontiguousarray(modes[b == i]).view([("", np.int64)] * 3).ravel())
        assert np.array_equal(ref, got), i
    # a subset of bins lists the same modes as the full listing restricted to them
    m2, b2 = shell_modes(n, thr, [3, 7])
    assert np.array_equal(np.sort(b2), np.sort(b[(b == 3) | (b == 7)]))


def _on_node_catalog(n, L, npart, seed, weights=True):
    rng = np.random.default_rng(seed)
    cells = rng.integers(0, n, size=(npart, 3))
    o = -0.5 * L
    pos = o + cells * (L / n)
    w = rng.uniform(0.5, 1.5, npart) if weights else np.ones(npart)
    return Catalog(pos, w, np.full(npart, npart / L ** 3))


@pytest.mark.parametrize("n", [16, 24])
def test_yamamoto_at_shell_modes_equals_fft_oracle_on_nodes(n):
    L = 200.0
    d = _on_node_catalog(n, L, 300, seed=n)
    p = default_params(n, L, observer=(13.0, -7.0, -400.0), window=1, interlaced=False, compensated=False)
    kf = 2 * math.pi / L
    edges = np.array([0.5, 1.5, 2.5, 3.5, math.sqrt(29.5), math.sqrt(30.5), math.sqrt(41.5), math.sqrt(42.5)]) * kf
    ells = [0, 2, 4, 6, 8]
    ref = multipoles(d, None, p, 8, edges)
    thr = k_thresholds(edges, L)
    sel = [0, 1, 2, 4, 6]      # the shells; bins 3 and 5 are the gaps between them
    modes, b = shell_modes(n, thr, sel)
    poles, counts, kmean = yamamoto_at_modes(d, None, p, ells, modes, b, thr.size - 1)
    assert np.array_equal(counts[sel].astype(np.int64), ref["n_modes"][sel])
    assert np.allclose(kmean[sel], ref["k_mean"][sel], rtol=1e-14, atol=0)
    scale = np.abs(ref["poles"][0][sel] + ref["shot_noise"])
    err = np.max(np.abs(poles[:, sel] - ref["poles"][:, sel]) / scale[None, :])
    assert err < 1e-12, err


@pytest.mark.parametrize("window", [1, 2, 3])
@pytest.mark.parametrize("interlaced,compensated", [(False, False), (True, True), (False, True)])
def test_combined_at_modes_equals_fft_combine(window, interlaced, compensated):
    n, L = 16, 150.0
    rng = np.random.default_rng(window + 10 * interlaced + 100 * compensated)
    d = Catalog(-L / 2 + rng.random((40, 3)) * L, rng.uniform(0.5, 1.5, 40), np.full(40, 40 / L ** 3))
    r = Catalog(-L / 2 + rng.random((160, 3)) * L, rng.uniform(0.5, 1.5, 160), np.full(160, 40 / L ** 3))
    p = default_params(n, L, window=window, interlaced=interlaced, compensated=compensated)
    _, c, _ = density_fields(d, r, p)
    f = int_freq(n)
    grid = np.stack(np.meshgrid(f, f, f, indexing="ij"), axis=-1).reshape(-1, 3)
    got = combined_at_modes(d, r, p, grid)
    assert np.max(np.abs(got - c.ravel())) < 1e-12 * np.max(np.abs(c))
    # Nyquist modes are zero on both sides
    nyq = np.any(grid == -(n // 2), axis=1)
    assert np.all(got[nyq] == 0)
