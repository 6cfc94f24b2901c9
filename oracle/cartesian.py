"""O4: the Cartesian decomposition (Sec. 2.1: Bianchi et al. 2015 / Scoccimarro 2015), FP64.

L_l(khat . xhat) is a polynomial in khat . xhat; multiplying each power (khat . xhat)^j by
(khat . khat)^((l-j)/2) (xhat . xhat)^((l-j)/2) = 1 makes it homogeneous of degree l in both
vectors, so  L_l(khat . xhat) = sum_{|a| = l} xhat^a g_a(khat)  and
A_l(n) = sum_{|a| = l} g_a(khat_n) DFT[D_c xhat^a](n):  (l+1)(l+2)/2 transforms per l.
"""
from __future__ import annotations

import math
from collections import defaultdict
from itertools import product

import numpy as np
import scipy.fft as sfft

from .estimator import density_fields, k_thresholds, mode_bins, node_vectors, mode_vectors, binned_sums
from .legendre import legendre_coefficients


def _compositions(total: int):
    for a in range(total + 1):
        for b in range(total - a + 1):
            yield (a, b, total - a - b)


def _multinom(p, parts):
    return math.factorial(p) // (math.factorial(parts[0]) * math.factorial(parts[1]) * math.factorial(parts[2]))


def _poly_mul(p, q):
    out = defaultdict(float)
    for (ka, ca) in p.items():
        for (kb, cb) in q.items():
            out[tuple(x + y for x, y in zip(ka, kb))] += ca * cb
    return dict(out)


def cartesian_terms(ell: int):
    """{x exponent a (|a| = l): {k exponent b: coeff}} for L_l(khat . xhat)."""
    coef = legendre_coefficients(ell)
    total = defaultdict(float)
    for j in range(ell + 1):
        if coef[j] == 0.0:
            continue
        p = (ell - j) // 2
        dot = {tuple(a) + tuple(a): float(_multinom(j, a)) for a in _compositions(j)}
        kk = {(0, 0, 0) + tuple(2 * x for x in a): float(_multinom(p, a)) for a in _compositions(p)}
        xx = {tuple(2 * x for x in a) + (0, 0, 0): float(_multinom(p, a)) for a in _compositions(p)}
        for key, val in _poly_mul(_poly_mul(dot, kk), xx).items():
            total[key] += coef[j] * val
    terms = defaultdict(dict)
    for key, val in total.items():
        if val != 0.0:
            terms[key[:3]][key[3:]] = val
    return dict(terms)


def _mono(vec, e):
    return vec[..., 0] ** e[0] * vec[..., 1] ** e[1] * vec[..., 2] ** e[2]


def cartesian_multipoles(data, randoms, params, ells, k_edges):
    n = params["nmesh"]
    L = params["box_len"]
    sc, c, dc = density_fields(data, randoms, params)
    thr = k_thresholds(k_edges, L)
    nb = thr.size - 1
    bins = mode_bins(n, thr)
    counts = binned_sums(np.ones(bins.shape), bins, nb)
    xv = node_vectors(n, L, params["box_origin"], params["observer"])
    xv = xv / np.sqrt(np.sum(xv * xv, axis=-1, keepdims=True))
    kv = mode_vectors(n)
    kr = np.sqrt(np.sum(kv * kv, axis=-1, keepdims=True))
    kv = kv / np.where(kr > 0, kr, 1.0)
    out = np.empty((len(ells), nb))
    nfft = 0
    for i, ell in enumerate(ells):
        if ell == 0:
            a = c
        else:
            a = np.zeros_like(c)
            for xe, kterms in cartesian_terms(ell).items():
                b = sfft.fftn(dc * _mono(xv, xe))
                nfft += 1
                g = np.zeros(c.shape)
                for ke, val in kterms.items():
                    g += val * _mono(kv, ke)
                a += g * b
        q = (2 * ell + 1) * np.real(c * np.conj(a))
        with np.errstate(invalid="ignore", divide="ignore"):
            out[i] = binned_sums(q, bins, nb) / (sc["norm_I"] * counts)
        if ell == 0:
            out[i] -= sc["shot_noise"]
    return out, counts, nfft


def cartesian_fft_count(ell_max: int) -> int:
    """Total transforms for all even l <= ell_max with the Cartesian method (Sec. 2.1)."""
    return sum((l + 1) * (l + 2) // 2 for l in range(0, ell_max + 1, 2))


def harmonic_fft_count(ell_max: int) -> int:
    """Total transforms for all even l <= ell_max with the harmonic method (Sec. 2.1)."""
    return sum(2 * l + 1 for l in range(0, ell_max + 1, 2))
