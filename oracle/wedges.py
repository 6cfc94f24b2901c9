"""Wedges from multipoles (Sec. 2.2, eq. wedge-est with eq. Lbar), FP64."""
from __future__ import annotations

import numpy as np

from .legendre import lbar


def lbar_matrix(ells, mu_edges) -> np.ndarray:
    """M[m, i] = Lbar_{ells[i]}(mu_m, mu_{m+1})."""
    e = np.asarray(mu_edges, dtype=np.float64)
    return np.stack([lbar(ell, e[:-1], e[1:]) for ell in ells], axis=1)


def wedges(poles, ells, mu_edges) -> np.ndarray:
    """P(k_i, mu_m) = sum_l P_l(k_i) Lbar_l(mu_m, mu_{m+1}); returns (n_k, n_mu)."""
    return np.asarray(poles, dtype=np.float64).T @ lbar_matrix(ells, mu_edges).T
