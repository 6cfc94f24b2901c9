"""Helpers of the cubic-box transverse-systematic test (Sec. 3.2), shared by the oracle pins and
the GPU tests.  They hold closed forms from the Legendre algebra, not the estimator."""
from __future__ import annotations

import numpy as np


def spike_edges(j, box_len):
    """One k bin holding exactly the modes with |n|^2 = j^2 (for j a power of two these are the
    six axis modes): edges (j -/+ 1/(4j)) k_f give thresholds ceil((j -/+ 1/(4j))^2) = j^2, j^2 + 1."""
    kf = 2.0 * np.pi / box_len
    return np.array([(j - 0.25 / j) * kf, (j + 0.25 / j) * kf])


def spike_decomposition(poles, shot_noise, ells):
    """With the line of sight along z everywhere, the modes (+-j,0,0), (0,+-j,0) sit at mu = 0 and
    (0,0,+-j) at mu = +-1, so every multipole of the spike bin is (2l+1)[a L_l(0) + b].  Fit a and
    b from l = 0, 2 and return them with the largest relative misfit over all l."""
    from numpy.polynomial import legendre as npl
    ells = np.asarray(ells)
    y = np.array(poles, dtype=np.float64)
    y[0] += shot_noise
    y /= 2 * ells + 1
    l0 = np.array([npl.legval(0.0, np.eye(l + 1)[l]) for l in ells])
    a = (y[0] - y[1]) / (l0[0] - l0[1])
    b = y[0] - a
    return a, b, float(np.max(np.abs(y - (a * l0 + b))) / abs(a))


def leakage_ratio_theory(lmax, mu_edges):
    """Spike in each wedge relative to the first: bin averages of the truncated delta series
    sum_l (2l+1) L_l(0) L_l(mu) = (lmax+1) L_lmax(0) L_{lmax+1}(mu)/mu (Christoffel, Sec. 3.1),
    integrated by Gauss-Legendre quadrature (the integrand is a polynomial)."""
    from numpy.polynomial import legendre as npl
    x, w = npl.leggauss(32)
    c = np.eye(lmax + 2)[lmax + 1]
    avg = []
    for lo, hi in zip(mu_edges[:-1], mu_edges[1:]):
        mu = 0.5 * (hi - lo) * x + 0.5 * (hi + lo)
        avg.append(0.5 * np.sum(w * npl.legval(mu, c) / mu))
    avg = np.array(avg)
    return avg / avg[0]
