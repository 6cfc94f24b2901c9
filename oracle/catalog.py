"""FKP normalisation scalars (Sec. 2.1, eq. FKP-density and the shot-noise term), FP64.

The paper defines F(r) = w [n - alpha n_s] / I^(1/2), I = int w^2 nbar^2 dr, and the
monopole shot noise (1 + alpha) int nbar w^2 (zero for l > 0).  Discrete readings:

* alpha = N_data / N_randoms (ratio of unweighted counts: the number-density ratio).
* I     = alpha * sum_randoms w^2 nbar       (randoms sample int dr with density nbar/alpha).
* S     = (sum_data w^2 + alpha^2 sum_randoms w^2) / I.
* Periodic box (no randoms): nbar = N_data / L^3, I = nbar sum_data w^2, S = sum_data w^2 / I
  (= 1/nbar for unit weights).
"""
from __future__ import annotations

import numpy as np


def _w(cat, n):
    return np.ones(n) if cat.w is None else np.asarray(cat.w, dtype=np.float64)


def catalog_scalars(data, randoms, box_len: float):
    """Return dict(alpha, norm_I, shot_noise) for a data catalog and optional randoms."""
    nd = data.pos.shape[0]
    wd = _w(data, nd)
    s_d2 = float(np.sum(wd * wd))
    if randoms is None:
        nbar = nd / box_len ** 3
        norm = nbar * s_d2
        return dict(alpha=0.0, norm_I=norm, shot_noise=s_d2 / norm)
    nr = randoms.pos.shape[0]
    if randoms.nbar is None:
        raise ValueError("randoms need nbar")
    wr = _w(randoms, nr)
    alpha = nd / nr
    norm = alpha * float(np.sum(wr * wr * np.asarray(randoms.nbar, dtype=np.float64)))
    shot = (s_d2 + alpha * alpha * float(np.sum(wr * wr))) / norm
    return dict(alpha=alpha, norm_I=norm, shot_noise=shot)
