"""Brute-force tiers of the oracle (tiny inputs only), FP64.

O1: the literal Legendre-weighted DFT of the mesh field (no spherical harmonics):
    A_l(n) = sum_c D_c(c) L_l(khat_n . xhat_c) exp(-2 pi i n.c / N).
    By the addition theorem (eq. add-theorem) this equals the harmonic form of eq. Fell.
O2: galaxy-direct Yamamoto sums (eq. Pell-yama) on the mesh's discrete modes:
    F_l(k) = sum_data w L_l(khat . rhat) exp(-i k.(r - o)) - alpha sum_rand w L_l(...) exp(...),
    P_l = (2l+1)/(I N_i) sum_bin Re[F_0 conj F_l] - delta_{l0} S,  with rhat from the observer.
    ``yamamoto_at_modes`` evaluates these sums over an explicit list of modes, so that only
    the modes of a few k bins (``shell_modes``, enumerated without the full grid) are needed
    on meshes whose full grid would not fit in host memory.
C at chosen modes (``combined_at_modes``): the combined, compensated transform of the
    painted meshes (Sec. 2.3) evaluated mode by mode as a direct sum over every painted tap,
    D~(n) = sum_taps w W exp(-2 pi i n.c / N), without a transform or a mesh.
"""
from __future__ import annotations

import math

import numpy as np

from .catalog import catalog_scalars
from .estimator import density_fields, k_thresholds, mode_bins, node_vectors, binned_sums, pole_term
from .legendre import legendre
from .mesh import axis_taps, compensation_1d, int_freq, mesh_coords


def _unit(v):
    r = np.sqrt(np.sum(v * v, axis=-1, keepdims=True))
    return v / np.where(r > 0, r, 1.0)


def _phase(modes, rel, box_len: float, sign: float = -1.0) -> np.ndarray:
    """exp(sign i k.rel) for k = 2 pi n / L, shape (modes, points).  The argument n.rel is
    formed and reduced modulo L in extended precision (long double) before the FP64
    exponential: formed in FP64, a product |n| |rel| ~ N L carries about N ulps of absolute
    error into the phase (1e-13 rad at N ~ 500), which the direct sums would then report as a
    difference from the mesh transform."""
    ld = np.longdouble
    t = np.asarray(modes, dtype=ld) @ np.asarray(rel, dtype=ld).T
    t = np.mod(t, ld(box_len))
    arg = (t * (ld(2.0) * ld(np.pi) / ld(box_len))).astype(np.float64)
    return np.exp(sign * 1j * arg)


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
        q = pole_term(ell, cf, a)
        with np.errstate(invalid="ignore", divide="ignore"):
            out[i] = binned_sums(q, bins, nb) / (sc["norm_I"] * counts)
        if ell == 0:
            out[i] -= sc["shot_noise"]
    return out, counts


def shell_modes(nmesh: int, thresholds: np.ndarray, bins) -> tuple:
    """Integer modes of the listed k bins: n with T_i <= |n|^2 < T_{i+1}, n != 0, and every
    component in [-N/2 + 1, N/2 - 1] (a component -N/2 puts a mode on a Nyquist plane, which
    belongs to no bin).  Enumerated over (n_x, n_y) with the n_z range solved in integers.
    Returns (modes (K, 3) int64, bin index (K,) int64), each full-sphere mode once."""
    h = nmesh // 2
    thr = np.asarray(thresholds, dtype=np.int64)
    a = np.arange(-h + 1, h, dtype=np.int64)
    ax, ay = np.meshgrid(a, a, indexing="ij")
    ax, ay = ax.ravel(), ay.ravel()
    s2 = ax * ax + ay * ay
    modes, which = [], []
    for b in bins:
        lo, hi = int(thr[b]), int(thr[b + 1])
        sel = s2 < hi
        px, py, ps = ax[sel], ay[sel], s2[sel]
        # largest z with z^2 <= hi - 1 - s2, smallest z >= 0 with z^2 >= lo - s2
        zmax = np.floor(np.sqrt((hi - 1 - ps).astype(np.float64))).astype(np.int64)
        zmax -= (zmax * zmax > hi - 1 - ps)
        zmax += ((zmax + 1) * (zmax + 1) <= hi - 1 - ps)
        need = np.maximum(lo - ps, 0)
        zmin = np.ceil(np.sqrt(need.astype(np.float64))).astype(np.int64)
        zmin += (zmin * zmin < need)
        zmin -= ((zmin > 0) & ((zmin - 1) * (zmin - 1) >= need))
        zmax = np.minimum(zmax, h - 1)
        keep = zmin <= zmax
        for x, y, z0, z1 in zip(px[keep], py[keep], zmin[keep], zmax[keep]):
            for z in range(int(z0), int(z1) + 1):
                for zz in ((z,) if z == 0 else (z, -z)):
                    if x == 0 and y == 0 and zz == 0:
                        continue
                    modes.append((x, y, zz))
                    which.append(b)
    if not modes:
        return np.zeros((0, 3), dtype=np.int64), np.zeros(0, dtype=np.int64)
    return np.array(modes, dtype=np.int64), np.array(which, dtype=np.int64)


def yamamoto_at_modes(data, randoms, params, ells, modes, bin_of, nb, chunk: int = 2048):
    """O2 per bin over the listed integer modes (each full-sphere mode once): returns
    (poles (len(ells), nb), counts (nb,), k_mean (nb,)); NaN where a bin has no mode."""
    L = params["box_len"]
    sc = catalog_scalars(data, randoms, L)
    o = np.asarray(params["box_origin"], dtype=np.float64)
    obs = np.asarray(params["observer"], dtype=np.float64)
    bins = np.asarray(bin_of, dtype=np.int64)
    counts = np.bincount(bins, minlength=nb).astype(np.float64)
    kmag = (2.0 * math.pi / L) * np.sqrt(np.sum(np.asarray(modes, np.float64) ** 2, axis=1))
    sums = np.zeros((len(ells), nb))
    cats = [(data, 1.0)] + ([(randoms, -sc["alpha"])] if randoms is not None else [])
    prep = []
    for cat, sgn in cats:
        w = np.ones(cat.pos.shape[0]) if cat.w is None else np.asarray(cat.w, np.float64)
        rel = np.asarray(cat.pos, dtype=np.longdouble) - np.asarray(o, dtype=np.longdouble)
        prep.append((rel, _unit(np.asarray(cat.pos, np.float64) - obs), sgn * w))
    want = sorted(set(ells) | {0})
    for s in range(0, len(modes), chunk):
        mchunk = np.asarray(modes[s:s + chunk])
        khat = _unit(mchunk.astype(np.float64))
        fl = {ell: np.zeros(len(mchunk), dtype=np.complex128) for ell in want}
        for rel, rhat, w in prep:
            ph = _phase(mchunk, rel, L)                             # (modes, particles)
            mu = khat @ rhat.T
            for ell in want:
                fl[ell] += ((ph * legendre(ell, mu)) if ell > 0 else ph) @ w
        b = bins[s:s + chunk]
        for i, ell in enumerate(ells):
            sums[i] += np.bincount(b, weights=pole_term(ell, fl[0], fl[ell]), minlength=nb)
    with np.errstate(invalid="ignore", divide="ignore"):
        poles = sums / (sc["norm_I"] * counts)
        kmean = np.bincount(bins, weights=kmag, minlength=nb) / counts
    for i, ell in enumerate(ells):
        if ell == 0:
            poles[i] -= sc["shot_noise"]
    return poles, counts, kmean


def yamamoto_direct(data, randoms, params, ells, k_edges):
    """O2 on the mesh's modes (all non-Nyquist n with a bin), exact particle positions."""
    n = params["nmesh"]
    L = params["box_len"]
    thr = k_thresholds(k_edges, L)
    nb = thr.size - 1
    bins = mode_bins(n, thr).ravel()
    f = int_freq(n)
    grid = np.stack(np.meshgrid(f, f, f, indexing="ij"), axis=-1).reshape(-1, 3)
    sel = bins >= 0
    poles, counts, _ = yamamoto_at_modes(data, randoms, params, ells, grid[sel], bins[sel], nb)
    return poles, counts


def pell_complex_literal(data, randoms, params, ell, modes, bin_of, nb, form: str = "ours"):
    """The shell average of the paper's estimator written out literally, as a complex number,
    for the listed modes, with F_l(k) = sum_data w L_l(khat . rhat) exp(+i k.r)
    - alpha sum_rand (...) (eq. Fell), rhat from the observer, each sum evaluated directly at
    the wave vector it needs (no conjugate symmetry used):
      form "ours": eq. Pell-ours, (2l+1)/(I N_i) sum_k F_0(k) F_l(-k);
      form "yama": eq. Pell-yama, (2l+1)/(I N_i) sum_k F_0(k) G_l(k),
                   G_l(k) = sum w L_l(khat . rhat) exp(-i k.r).
    Even l: both are real, P_l + delta_l0 S.  Odd l: the real part vanishes; "ours" gives
    i R_l and "yama" -i R_l (step 7 of the FFT oracle)."""
    L = params["box_len"]
    sc = catalog_scalars(data, randoms, L)
    obs = np.asarray(params["observer"], dtype=np.float64)
    m = np.asarray(modes, dtype=np.int64)

    def F(ell, mv, sign):
        khat = _unit(mv.astype(np.float64))
        v = np.zeros(len(mv), dtype=np.complex128)
        for cat, sgn in ((data, 1.0), (randoms, -sc["alpha"])):
            if cat is None:
                continue
            pos = np.asarray(cat.pos, dtype=np.float64)
            w = sgn * (np.ones(pos.shape[0]) if cat.w is None else np.asarray(cat.w, np.float64))
            lw = legendre(ell, khat @ _unit(pos - obs).T) if ell > 0 else 1.0
            v += (_phase(mv, pos, L, sign) * lw) @ w
        return v

    if form == "ours":
        prod = F(0, m, 1) * F(ell, -m, 1)
    elif form == "yama":
        prod = F(0, m, 1) * F(ell, m, -1)
    else:
        raise ValueError("form must be 'ours' or 'yama'")
    b = np.asarray(bin_of, dtype=np.int64)
    counts = np.bincount(b, minlength=nb).astype(np.float64)
    re = np.bincount(b, weights=prod.real, minlength=nb)
    im = np.bincount(b, weights=prod.imag, minlength=nb)
    with np.errstate(invalid="ignore", divide="ignore"):
        return (2 * ell + 1) * (re + 1j * im) / (sc["norm_I"] * counts)


def combined_at_modes(data, randoms, params, modes) -> np.ndarray:
    """C(n) at the listed integer modes (components in [-N/2, N/2)): for each painted mesh,
    D~(n) = sum over particles and taps of w W exp(-2 pi i n.c / N) with c the tap's node
    (the unwrapped index gives the same phase); C = [D1~ + exp(+i pi (n_x+n_y+n_z)/N) D2~] / 2
    when interlaced (D2 painted at u + 1/2), else D1~; divided by W_c when compensated; zero
    when a component equals -N/2."""
    n = params["nmesh"]
    L = params["box_len"]
    window = params["window"]
    sc = catalog_scalars(data, randoms, L)
    m = np.asarray(modes, dtype=np.int64)
    mf = m.astype(np.float64)

    def dft(shift):
        v = np.zeros(len(m), dtype=np.complex128)
        for cat, sgn in ((data, 1.0), (randoms, -sc["alpha"])):
            if cat is None:
                continue
            u = mesh_coords(cat.pos, L, params["box_origin"], n)
            if shift:
                u = u + 0.5
            w = sgn * (np.ones(cat.pos.shape[0]) if cat.w is None else np.asarray(cat.w, np.float64))
            tx, ty, tz = axis_taps(u[:, 0], window), axis_taps(u[:, 1], window), axis_taps(u[:, 2], window)
            for ix, wx in tx:
                for iy, wy in ty:
                    for iz, wz in tz:
                        node = np.stack([ix, iy, iz], axis=1)                      # (particles, 3) ints
                        red = np.mod(m @ node.T, n)                                # n.c mod N, exact
                        ph = np.exp(-2j * math.pi * red / n)                       # (modes, particles)
                        v += ph @ (w * wx * wy * wz)
        return v

    c = dft(False)
    if params["interlaced"]:
        phi = np.exp(1j * math.pi * mf.sum(axis=1) / n)
        c = 0.5 * (c + phi * dft(True))
    if params["compensated"]:
        w1 = compensation_1d(n, window, params["interlaced"])
        idx = np.mod(m, n)
        c = c / (w1[idx[:, 0]] * w1[idx[:, 1]] * w1[idx[:, 2]])
    c[np.any(m == -(n // 2), axis=1)] = 0.0
    return c
