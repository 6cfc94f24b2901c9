"""Brute-force tiers of the oracle (tiny inputs only), FP64.

O1: the literal Legendre-weighted DFT of the mesh field (no spherical harmonics):
    A_l(n) = sum_c D_c(c) L_l(khat_n . xhat_c) exp(-2 pi i n.c / N).
    By the addition theorem (eq. add-theorem) this equals the harmonic form of eq. Fell.
O2: galaxy-direct Yamamoto sums (eq. Pell-yama) on the mesh's discrete modes:
    F_l(k) = sum_data w L_l(khat . rhat) exp(-i k.(r - o)) - alpha sum_rand w L_l(...) exp(...),
    P_l = (2l+1)/(I N_i) sum_bin Re[F_0 conj F_l] - delta_{l0} S,  with rhat from the observer.
"""
from __future__ import annotations

import math

import numpy as np

from .catalog import catalog_scalars
from .estimator import density_fields, k_thresholds, mode_bins, node_vectors, binned_sums
from .legendre import legendre
from .mesh import int_freq


def _unit(v):
    r = np.sqrt(np.sum(v * v, axis=-1, keepdims=True))
    return v / np.where(r > 0, r, 1.0)


def brute_force_multipoles(data, randoms, params, ells, k_edges):
    """O1 over the full grid; cost O(N^6) per l, so N <= 16."""
    n = params["nmesh"]
    L = params["box_len"]
    sc, c, dc = density_fields(data, randoms, params)
    thr = k_thresholds(k_edges, L)
    nb = thr.size - 1
    bins = mode_bins(n, thr).ravel()
    counts = binned_sums(np.ones(bins.shape), bins, nb)
    f = int_freq(n)
    grid = np.stack(np.meshgrid(f, f, f, indexing="ij"), axis=-1).reshape(-1, 3)
    idx = np.arange(n)
    nodes = np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), axis=-1).reshape(-1, 3)
    xhat = _unit(node_vectors(n, L, params["box_origin"], params["observer"]).reshape(-1, 3))
    khat = _unit(grid.astype(np.float64))
    phase = np.exp(-2j * math.pi * (grid @ nodes.T) / n)           # (modes, nodes)
    dcf = dc.ravel()
    cf = c.ravel()
    out = np.empty((len(ells), nb))
    for i, ell in enumerate(ells):
        lw = legendre(ell, khat @ xhat.T)                          # (modes, nodes)
        a = (phase * lw) @ dcf
        q = (2 * ell + 1) * np.real(cf * np.conj(a))
        with np.errstate(invalid="ignore", divide="ignore"):
            out[i] = binned_sums(q, bins, nb) / (sc["norm_I"] * counts)
        if ell == 0:
            out[i] -= sc["shot_noise"]
    return out, counts


def yamamoto_direct(data, randoms, params, ells, k_edges):
    """O2 on the mesh's modes (all non-Nyquist n with a bin), exact particle positions."""
    n = params["nmesh"]
    L = params["box_len"]
    sc = catalog_scalars(data, randoms, L)
    thr = k_thresholds(k_edges, L)
    nb = thr.size - 1
    bins = mode_bins(n, thr).ravel()
    f = int_freq(n)
    grid = np.stack(np.meshgrid(f, f, f, indexing="ij"), axis=-1).reshape(-1, 3)
    sel = bins >= 0
    grid = grid[sel]
    bsel = bins[sel]
    counts = np.bincount(bsel, minlength=nb).astype(np.float64)
    kvec = grid.astype(np.float64) * (2.0 * math.pi / L)
    khat = _unit(kvec)
    o = np.asarray(params["box_origin"], dtype=np.float64)
    obs = np.asarray(params["observer"], dtype=np.float64)

    def field(cat, sign_alpha, ell):
        w = np.ones(cat.pos.shape[0]) if cat.w is None else np.asarray(cat.w, np.float64)
        rhat = _unit(cat.pos - obs)
        ph = np.exp(-1j * (kvec @ (cat.pos - o).T))                # (modes, particles)
        lw = legendre(ell, khat @ rhat.T) if ell > 0 else 1.0
        return sign_alpha * ((ph * lw) @ w)

    def fl(ell):
        v = field(data, 1.0, ell)
        if randoms is not None:
            v = v + field(randoms, -sc["alpha"], ell)
        return v

    f0 = fl(0)
    out = np.empty((len(ells), nb))
    for i, ell in enumerate(ells):
        q = (2 * ell + 1) * np.real(f0 * np.conj(fl(ell)))
        with np.errstate(invalid="ignore", divide="ignore"):
            out[i] = np.bincount(bsel, weights=q, minlength=nb) / (sc["norm_I"] * counts)
        if ell == 0:
            out[i] -= sc["shot_noise"]
    return out, counts
