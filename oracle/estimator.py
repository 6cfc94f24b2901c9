"""O3: the spherical-harmonic FFT estimator on the mesh (Sec. 2.1, eq. Pell-ours, eq. Fell),
in FP64 with scipy.fft.  This is the oracle used at workload sizes.

Definition followed, step by step (conventions in ``oracle/__init__.py``):

1. alpha, I, S from the catalogs (``catalog.catalog_scalars``).
2. D1 (and D2 when interlaced) painted on the mesh (``mesh.fkp_meshes``).
3. C = combined, compensated forward transform with the Nyquist planes zeroed
   (``mesh.combine``).  C is F_0 of eq. Pell-ours on the mesh (up to I^(1/2)).
4. D_c = inverse transform of C (real part, 1/N^3 included).  When the mesh is neither
   interlaced nor compensated, D_c = D1 directly (no transform pair is needed).
5. For even l > 0:  A_l(n) = 4 pi/(2l+1) sum_m Y_lm(khat_n) DFT[D_c Y_lm(xhat_c)](n)
   (eq. Fell with the real harmonics of eq. real-Ylm; xhat_c is the unit vector from the
   observer to node c, khat_n = n/|n|).  A_0 = C.
6. P_l(k_i) = (2l+1)/(I N_i) sum_{n in bin i} Re[C(n) conj(A_l(n))] - delta_{l0} S, over the
   full grid (each mode once), bin i = {T_i <= |n|^2 < T_{i+1}}, T_i = ceil((e_i L/2pi)^2),
   n = 0 and Nyquist-plane modes excluded; k_mean_i = mean of (2 pi/L)|n| over the bin.
7. Odd l (asked for through ``ells``): the shell average of eq. Pell-ours is purely
   imaginary, because a mode and its mirror -n contribute with L_l(-x) = -L_l(x) and their
   real parts cancel.  The oracle returns the real number
   R_l(k_i) = (2l+1)/(I N_i) sum_{n in bin i} Im[C(n) conj(A_l(n))], no shot-noise term.
   With the exponent exp(-i k.x) used here for C and A_l and the paper's exp(+i k.r) in
   eq. Fell, the complex multipole of eq. Pell-ours is i R_l, so R_l = Im P_l.  (Eq. Pell-yama,
   whose second integral is the complex conjugate of F_l(k) rather than F_l(-k), agrees with
   eq. Pell-ours for even l and has the opposite sign for odd l.)
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft

from .catalog import catalog_scalars
from .mesh import combine, fkp_meshes, int_freq, nyquist_mask
from .ylm import real_ylm


def k_thresholds(k_edges, box_len: float) -> np.ndarray:
    """T_i = ceil(t_i^2), t_i = (e_i * L) / (2 pi), in float64 in this operation order."""
    twopi = 2.0 * math.pi
    t = (np.asarray(k_edges, dtype=np.float64) * box_len) / twopi
    return np.ceil(t * t).astype(np.int64)


def mode_bins(nmesh: int, thresholds: np.ndarray) -> np.ndarray:
    """Bin index of every full-grid mode (FFT order), -1 where the mode is in no bin."""
    f = int_freq(nmesh)
    n2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2
    idx = np.searchsorted(thresholds, n2, side="right") - 1
    nb = thresholds.size - 1
    valid = (idx >= 0) & (idx < nb) & (n2 > 0) & nyquist_mask(nmesh)
    return np.where(valid, idx, -1)


def node_vectors(nmesh: int, box_len: float, origin, observer) -> np.ndarray:
    """x_c - observer for every node c (shape N,N,N,3), node c at o + c H."""
    h = box_len / nmesh
    c = np.arange(nmesh, dtype=np.float64)
    o = np.asarray(origin, dtype=np.float64)
    obs = np.asarray(observer, dtype=np.float64)
    out = np.empty((nmesh, nmesh, nmesh, 3))
    out[..., 0] = (o[0] + c * h - obs[0])[:, None, None]
    out[..., 1] = (o[1] + c * h - obs[1])[None, :, None]
    out[..., 2] = (o[2] + c * h - obs[2])[None, None, :]
    return out


def mode_vectors(nmesh: int) -> np.ndarray:
    f = int_freq(nmesh).astype(np.float64)
    out = np.empty((nmesh, nmesh, nmesh, 3))
    out[..., 0] = f[:, None, None]
    out[..., 1] = f[None, :, None]
    out[..., 2] = f[None, None, :]
    return out


def binned_sums(values: np.ndarray, bins: np.ndarray, nbins: int) -> np.ndarray:
    sel = bins >= 0
    return np.bincount(bins[sel], weights=values[sel], minlength=nbins)


def density_fields(data, randoms, params, workers: int = 1):
    """Steps 1-4: scalars, C (full grid) and D_c."""
    n = params["nmesh"]
    L = params["box_len"]
    sc = catalog_scalars(data, randoms, L)
    d1, d2 = fkp_meshes(data, randoms, sc["alpha"], n, L, params["box_origin"],
                        params["window"], params["interlaced"])
    c = combine(d1, d2, n, params["window"], params["interlaced"], params["compensated"], workers)
    if params["interlaced"] or params["compensated"]:
        dc = sfft.ifftn(c, workers=workers).real
    else:
        dc = d1
    return sc, c, dc


def field_multipole(c: np.ndarray, dc: np.ndarray, ell: int, params, xvec=None, kvec=None,
                    workers: int = 1) -> np.ndarray:
    """A_l(n) on the full grid (step 5)."""
    if ell == 0:
        return c
    n = params["nmesh"]
    if xvec is None:
        xvec = node_vectors(n, params["box_len"], params["box_origin"], params["observer"])
    if kvec is None:
        kvec = mode_vectors(n)
    a = np.zeros_like(c)
    for m in range(-ell, ell + 1):
        b = sfft.fftn(dc * real_ylm(ell, m, xvec), workers=workers)
        a += real_ylm(ell, m, kvec) * b
    return a * (4.0 * math.pi / (2 * ell + 1))


def pole_term(ell: int, c: np.ndarray, a: np.ndarray) -> np.ndarray:
    """(2l+1) Re[C conj A_l] for even l, (2l+1) Im[C conj A_l] for odd l (steps 6 and 7)."""
    z = c * np.conj(a)
    return (2 * ell + 1) * (np.imag(z) if ell % 2 else np.real(z))


def multipoles(data, randoms, params, ell_max: int, k_edges, workers: int = 1, ells=None):
    """P_l(k) for even l <= ell_max (or the listed ``ells``, odd ones giving R_l of step 7).
    Returns dict with poles (n_ell, n_k), k_mean, n_modes, alpha, norm_I, shot_noise and
    n_transforms."""
    if ells is None and (ell_max % 2 or ell_max < 0):
        raise ValueError("ell_max must be even and >= 0")
    n = params["nmesh"]
    L = params["box_len"]
    ells = list(range(0, ell_max + 1, 2)) if ells is None else list(ells)
    sc, c, dc = density_fields(data, randoms, params, workers)
    thr = k_thresholds(k_edges, L)
    nb = thr.size - 1
    bins = mode_bins(n, thr)
    counts = binned_sums(np.ones(bins.shape), bins, nb)
    f = int_freq(n).astype(np.float64)
    kmag = (2.0 * math.pi / L) * np.sqrt(f[:, None, None] ** 2 + f[None, :, None] ** 2
                                         + f[None, None, :] ** 2)
    with np.errstate(invalid="ignore", divide="ignore"):
        kmean = binned_sums(kmag, bins, nb) / counts
    xvec = kvec = None
    if any(e > 0 for e in ells):
        xvec = node_vectors(n, L, params["box_origin"], params["observer"])
        kvec = mode_vectors(n)
    poles = np.empty((len(ells), nb))
    for i, ell in enumerate(ells):
        a = field_multipole(c, dc, ell, params, xvec, kvec, workers)
        q = pole_term(ell, c, a)
        with np.errstate(invalid="ignore", divide="ignore"):
            poles[i] = binned_sums(q, bins, nb) / (sc["norm_I"] * counts)
        if ell == 0:
            poles[i] -= sc["shot_noise"]
    n_fields = sum(2 * e + 1 for e in ells if e > 0)
    n_fwd = 2 if params["interlaced"] else 1
    n_inv = 1 if (params["interlaced"] or params["compensated"]) else 0
    return dict(poles=poles, ells=ells, k_mean=kmean, n_modes=counts.astype(np.int64),
                n_transforms=n_fields + n_fwd + n_inv, **sc)


def all_multipoles(data, randoms, params, ell_max: int, k_edges, workers: int = 1):
    """Every l = 0 .. ell_max: even rows P_l, odd rows R_l (step 7)."""
    return multipoles(data, randoms, params, ell_max, k_edges, workers, ells=list(range(ell_max + 1)))


def default_params(nmesh, box_len, observer=(0.0, 0.0, -1500.0), window=3, interlaced=True,
                   compensated=True, box_origin=None):
    o = (-0.5 * box_len,) * 3 if box_origin is None else tuple(box_origin)
    return dict(nmesh=int(nmesh), box_len=float(box_len), box_origin=o, observer=tuple(observer),
                window=int(window), interlaced=bool(interlaced), compensated=bool(compensated))


def default_k_edges(nmesh: int, box_len: float, dk: float = 0.01) -> np.ndarray:
    """Uniform edges e_i = i dk for i = 0 .. floor(k_N / dk), k_N = pi N / L."""
    kn = math.pi * nmesh / box_len
    nb = int(math.floor(kn / dk))
    return np.arange(nb + 1, dtype=np.float64) * dk
