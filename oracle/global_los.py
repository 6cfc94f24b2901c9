"""Fixed (global) line-of-sight statistics on the mesh, FP64.

With one LOS unit vector lhat for every pair, the multipoles reduce to
P_l(k) = (2l+1)/(I N_i) sum |C|^2 L_l(mu) - delta_{l0} S with mu = |khat . lhat|; the local
estimator tends to this when the observer recedes along -lhat (Sec. 1, plane-parallel
limit).  P(k, mu) bins the same |C|^2 in (k, mu) cells; mu bins are left-closed and
mu = 1 belongs to the last bin (Sec. 2.2 allows non-uniform mu edges).
"""
from __future__ import annotations

import numpy as np

from .estimator import density_fields, k_thresholds, mode_bins, binned_sums
from .legendre import legendre
from .mesh import int_freq


def mode_mu(nmesh: int, los) -> np.ndarray:
    """mu = |n . lhat| / |n| (0 at n = 0), float64 in this operation order."""
    l = np.asarray(los, dtype=np.float64)
    f = int_freq(nmesh).astype(np.float64)
    dot = (f[:, None, None] * l[0] + f[None, :, None] * l[1]) + f[None, None, :] * l[2]
    n2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2
    r = np.sqrt(n2)
    return np.where(n2 > 0, np.abs(dot) / np.where(n2 > 0, r, 1.0), 0.0)


def mu_bins(mu: np.ndarray, mu_edges) -> np.ndarray:
    e = np.asarray(mu_edges, dtype=np.float64)
    j = np.searchsorted(e, mu, side="right") - 1
    nm = e.size - 1
    j = np.where(mu >= e[-1], nm - 1, j)
    return np.where((j >= 0) & (j < nm), j, -1)


def pkmu(data, randoms, params, k_edges, mu_edges, los):
    """P(k_i, mu_j) and mode counts, arrays of shape (n_k, n_mu)."""
    n = params["nmesh"]
    sc, c, _ = density_fields(data, randoms, params)
    kb = mode_bins(n, k_thresholds(k_edges, params["box_len"]))
    mb = mu_bins(mode_mu(n, los), mu_edges)
    nk = len(k_edges) - 1
    nm = len(mu_edges) - 1
    cell = np.where((kb >= 0) & (mb >= 0), kb * nm + mb, -1)
    p2 = np.abs(c) ** 2
    cnt = binned_sums(np.ones(cell.shape), cell, nk * nm).reshape(nk, nm)
    s = binned_sums(p2, cell, nk * nm).reshape(nk, nm)
    with np.errstate(invalid="ignore", divide="ignore"):
        p = s / (sc["norm_I"] * cnt) - sc["shot_noise"]
    return p, cnt.astype(np.int64)


def global_multipoles(data, randoms, params, ells, k_edges, los):
    n = params["nmesh"]
    sc, c, _ = density_fields(data, randoms, params)
    kb = mode_bins(n, k_thresholds(k_edges, params["box_len"]))
    nk = len(k_edges) - 1
    mu = mode_mu(n, los)
    cnt = binned_sums(np.ones(kb.shape), kb, nk)
    p2 = np.abs(c) ** 2
    out = np.empty((len(ells), nk))
    for i, ell in enumerate(ells):
        with np.errstate(invalid="ignore", divide="ignore"):
            out[i] = (2 * ell + 1) * binned_sums(p2 * legendre(ell, mu), kb, nk) / (sc["norm_I"] * cnt)
        if ell == 0:
            out[i] -= sc["shot_noise"]
    return out, cnt
