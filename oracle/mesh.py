"""Mass assignment, interlacing and window compensation on an N^3 mesh (Sec. 2.3), FP64.

The paper paints with TSC on two meshes offset by half a cell, combines them in Fourier
space and corrects the assignment window (Jing 2005).  It fixes no formulas, so:

* Mesh coordinate of a position x: u = (x - o) * (N / L), node c at o + c H.
* NGP: node floor(u + 1/2), weight 1.
  CIC: nodes floor(u) + {0, 1}, weights (1 - d, d) with d = u - floor(u).
  TSC: nodes c + {-1, 0, 1} with c = floor(u + 1/2), d = u - c, weights
       (1/2 - d)^2 / 2, 3/4 - d^2, (1/2 + d)^2 / 2.
  The 3D weight is the product over axes; node indices wrap modulo N.
* Interlacing: the second mesh is painted at u + 1/2 on every axis.  The combined
  transform is C = [D1~ + phi D2~] / 2 with phi(n) = exp(+i pi (n_x + n_y + n_z) / N)
  (the average of the two aligned transforms).
* Compensation: interlaced -> W_c = prod_a sinc(pi n_a / N)^p (p = 1, 2, 3 for NGP, CIC,
  TSC).  Not interlaced -> W_c = prod_a sqrt(A_p(s_a)), s = sin(pi n_a / N), with the
  alias sums A_1 = 1, A_2 = 1 - 2 s^2 / 3, A_3 = 1 - s^2 + 2 s^4 / 15.  C is divided by W_c.
* Every mode with some n_a = -N/2 (the Nyquist planes) is set to zero in C.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

NGP, CIC, TSC = 1, 2, 3


def mesh_coords(pos: np.ndarray, box_len: float, origin, nmesh: int) -> np.ndarray:
    """u = (x - o) * (N / L) in float64 (this exact operation order)."""
    scale = nmesh / box_len
    return (np.asarray(pos, dtype=np.float64) - np.asarray(origin, dtype=np.float64)) * scale


def axis_taps(u: np.ndarray, window: int):
    """Per-axis node indices (unwrapped) and weights: lists of (idx, w) arrays."""
    if window == NGP:
        c = np.floor(u + 0.5)
        return [(c.astype(np.int64), np.ones_like(u))]
    if window == CIC:
        c = np.floor(u)
        d = u - c
        ci = c.astype(np.int64)
        return [(ci, 1.0 - d), (ci + 1, d)]
    if window == TSC:
        c = np.floor(u + 0.5)
        d = u - c
        ci = c.astype(np.int64)
        return [(ci - 1, 0.5 * (0.5 - d) ** 2), (ci, 0.75 - d * d), (ci + 1, 0.5 * (0.5 + d) ** 2)]
    raise ValueError("window must be 1 (NGP), 2 (CIC) or 3 (TSC)")


def paint(u: np.ndarray, weight: np.ndarray, nmesh: int, window: int) -> np.ndarray:
    """Sum over particles of weight * W(u - node) onto an nmesh^3 float64 mesh."""
    n = nmesh
    out = np.zeros(n * n * n)
    tx = axis_taps(u[:, 0], window)
    ty = axis_taps(u[:, 1], window)
    tz = axis_taps(u[:, 2], window)
    for ix, wx in tx:
        for iy, wy in ty:
            for iz, wz in tz:
                flat = ((ix % n) * n + (iy % n)) * n + (iz % n)
                out += np.bincount(flat, weights=weight * wx * wy * wz, minlength=n ** 3)
    return out.reshape(n, n, n)


def window_1d(d: np.ndarray, window: int) -> np.ndarray:
    """Assignment weight of a particle at signed distance d (in cells) from a node, written
    as the kernel itself rather than as taps: NGP 1 on [-1/2, 1/2); CIC max(0, 1 - |d|);
    TSC 3/4 - d^2 for |d| <= 1/2, (3/2 - |d|)^2 / 2 for 1/2 < |d| < 3/2, else 0."""
    a = np.abs(d)
    if window == NGP:
        return ((d >= -0.5) & (d < 0.5)).astype(np.float64)
    if window == CIC:
        return np.maximum(0.0, 1.0 - a)
    if window == TSC:
        return np.where(a <= 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))
    raise ValueError("window must be 1 (NGP), 2 (CIC) or 3 (TSC)")


def paint_at(u: np.ndarray, weight: np.ndarray, nmesh: int, window: int, cells: np.ndarray) -> np.ndarray:
    """Value of the painted mesh at the listed nodes (cells: (K, 3) ints): for each node c,
    sum over particles of weight * prod_a W(u_a - c_a), the distance wrapped to [-N/2, N/2).
    Same quantity as paint() at those nodes, evaluated from the kernel's definition."""
    u = np.asarray(u, dtype=np.float64)
    out = np.empty(len(cells))
    for i, c in enumerate(np.asarray(cells)):
        d = u - c[None, :]
        d = d - nmesh * np.floor(d / nmesh + 0.5)
        w = window_1d(d[:, 0], window) * window_1d(d[:, 1], window) * window_1d(d[:, 2], window)
        out[i] = np.sum(weight * w)
    return out


def fkp_meshes(data, randoms, alpha: float, nmesh: int, box_len: float, origin, window: int,
               interlaced: bool):
    """D1 (and D2 when interlaced) = sum_d w W - alpha sum_r w W."""
    def one(shift):
        ud = mesh_coords(data.pos, box_len, origin, nmesh)
        if shift:
            ud = ud + 0.5
        wd = np.ones(data.pos.shape[0]) if data.w is None else np.asarray(data.w, np.float64)
        d = paint(ud, wd, nmesh, window)
        if randoms is not None:
            ur = mesh_coords(randoms.pos, box_len, origin, nmesh)
            if shift:
                ur = ur + 0.5
            wr = np.ones(randoms.pos.shape[0]) if randoms.w is None else np.asarray(randoms.w, np.float64)
            d -= alpha * paint(ur, wr, nmesh, window)
        return d
    d1 = one(False)
    d2 = one(True) if interlaced else None
    return d1, d2


def int_freq(nmesh: int) -> np.ndarray:
    """Integer frequencies in FFT order: 0, 1, ..., N/2-1, -N/2, ..., -1."""
    return np.fft.fftfreq(nmesh, d=1.0 / nmesh).round().astype(np.int64)


def compensation_1d(nmesh: int, window: int, interlaced: bool) -> np.ndarray:
    """Per-axis factor of W_c(n) in FFT order."""
    n = int_freq(nmesh).astype(np.float64)
    x = np.pi * n / nmesh
    if interlaced:
        sinc = np.where(n == 0, 1.0, np.sin(x) / np.where(n == 0, 1.0, x))
        return sinc ** window
    s2 = np.sin(x) ** 2
    if window == NGP:
        a = np.ones_like(s2)
    elif window == CIC:
        a = 1.0 - 2.0 / 3.0 * s2
    else:
        a = 1.0 - s2 + 2.0 / 15.0 * s2 * s2
    return np.sqrt(a)


def nyquist_mask(nmesh: int) -> np.ndarray:
    """True where no component equals -N/2 (full grid, FFT order)."""
    f = int_freq(nmesh)
    ok = f != -(nmesh // 2)
    return ok[:, None, None] & ok[None, :, None] & ok[None, None, :]


def combine(d1: np.ndarray, d2, nmesh: int, window: int, interlaced: bool, compensated: bool,
            workers: int = 1) -> np.ndarray:
    """Full-grid complex C(n) (FFT order along every axis)."""
    c = sfft.fftn(d1, workers=workers)
    if interlaced:
        f = int_freq(nmesh).astype(np.float64)
        ph = np.exp(1j * np.pi * f / nmesh)
        phi = ph[:, None, None] * ph[None, :, None] * ph[None, None, :]
        c = 0.5 * (c + phi * sfft.fftn(d2, workers=workers))
    if compensated:
        w1 = compensation_1d(nmesh, window, interlaced)
        c /= w1[:, None, None] * w1[None, :, None] * w1[None, None, :]
    c[~nyquist_mask(nmesh)] = 0.0
    return c
