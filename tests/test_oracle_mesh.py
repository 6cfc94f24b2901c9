"""Pins of the oracle's mesh steps: painting, interlacing, compensation, transform sign."""
import math

import numpy as np
import pytest
import scipy.fft as sfft

from synth import Catalog
from oracle.catalog import catalog_scalars
from oracle.mesh import (CIC, NGP, TSC, axis_taps, combine, compensation_1d, fkp_meshes,
                         int_freq, mesh_coords, nyquist_mask, paint, paint_at, window_1d)


def _cat(pos, w=None, nbar=None):
    pos = np.atleast_2d(np.asarray(pos, dtype=np.float64))
    return Catalog(pos, None if w is None else np.asarray(w, float), None if nbar is None else np.asarray(nbar, float))


def test_catalog_scalars_hand_values():
    """alpha = N_d/N_r, I = alpha sum_r w^2 nbar, S = (sum_d w^2 + alpha^2 sum_r w^2)/I,
    evaluated by hand for a 2-galaxy / 4-random catalog."""
    d = _cat(np.zeros((2, 3)), w=[1.0, 2.0])
    r = _cat(np.zeros((4, 3)), w=[1.0, 1.0, 1.0, 1.0], nbar=[0.5, 0.5, 0.5, 0.5])
    sc = catalog_scalars(d, r, 10.0)
    assert sc["alpha"] == 0.5
    assert sc["norm_I"] == 1.0          # 0.5 * 4 * 0.5
    assert sc["shot_noise"] == 6.0      # (1 + 4 + 0.25 * 4) / 1
    p = catalog_scalars(_cat(np.zeros((8, 3))), None, 2.0)   # nbar = 1, I = 8
    assert p["norm_I"] == 8.0 and p["shot_noise"] == 1.0


@pytest.mark.parametrize("window", [NGP, CIC, TSC])
def test_partition_of_unity_and_mass(window):
    rng = np.random.default_rng(5)
    n, L = 16, 50.0
    pos = -L / 2 + rng.random((300, 3)) * L
    w = rng.uniform(0.5, 1.5, 300)
    u = mesh_coords(pos, L, (-L / 2,) * 3, n)
    for i in range(5):
        m = paint(u[i:i + 1], w[i:i + 1], n, window)
        assert abs(m.sum() - w[i]) < 1e-15 * 8
    d = _cat(pos[:100], w[:100])
    r = _cat(pos[100:], w[100:], np.ones(200))
    alpha = 100 / 200
    d1, d2 = fkp_meshes(d, r, alpha, n, L, (-L / 2,) * 3, window, True)
    ref = w[:100].sum() - alpha * w[100:].sum()
    assert abs(d1.sum() - ref) < 1e-12 and abs(d2.sum() - ref) < 1e-12


def test_on_node_stencils_and_wrap():
    n = 8
    u = np.array([[3.0, 0.0, 7.0]])
    m = paint(u, np.ones(1), n, CIC)
    assert m[3, 0, 7] == 1.0 and np.count_nonzero(m) == 1          # CIC on a node is a delta
    m = paint(u, np.ones(1), n, TSC)                                # TSC on a node: (1/8, 3/4, 1/8)^3
    s = np.array([0.125, 0.75, 0.125])
    ref = np.zeros((n, n, n))
    for a, ia in enumerate([2, 3, 4]):
        for b, ib in enumerate([7, 0, 1]):          # wraps across the y = 0 face
            for c, ic in enumerate([6, 7, 0]):      # and the z = N face
                ref[ia, ib, ic] += s[a] * s[b] * s[c]
    assert np.max(np.abs(m - ref)) < 1e-16
    # round-half-up tie break: u = 2.5 has TSC centre 3 and d = -1/2 -> weights (1/2, 1/2, 0)
    taps = axis_taps(np.array([2.5]), TSC)
    assert [int(t[0][0]) for t in taps] == [2, 3, 4]
    assert [float(t[1][0]) for t in taps] == [0.5, 0.5, 0.0]
    assert [int(t[0][0]) for t in axis_taps(np.array([2.5]), NGP)] == [3]


def test_forward_transform_convention():
    """scipy's fftn is the sum_c D(c) exp(-2 pi i n.c / N) assumed by the definition."""
    n = 6
    d = np.random.default_rng(1).normal(size=(n, n, n))
    c = np.arange(n)
    idx = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1).reshape(-1, 3)
    f = int_freq(n)
    modes = np.stack(np.meshgrid(f, f, f, indexing="ij"), -1).reshape(-1, 3)
    direct = np.exp(-2j * math.pi * (modes @ idx.T) / n) @ d.ravel()
    assert np.max(np.abs(direct - sfft.fftn(d).ravel())) < 1e-12


@pytest.mark.parametrize("window", [CIC, TSC])
def test_interlaced_single_particle_closed_form(window):
    """A unit particle on node p, interlaced, uncompensated: C(n) = 1/2 [A(n) + prod cos(k_a H/2)]
    e^{-i k.p} with A = 1 (CIC) or prod(3/4 + cos(k_a H)/4) (TSC), off the Nyquist planes."""
    n, L = 8, 8.0
    p = np.array([2, 5, 1])
    d = _cat(-L / 2 + p * (L / n))
    d1, d2 = fkp_meshes(d, None, 0.0, n, L, (-L / 2,) * 3, window, True)
    c = combine(d1, d2, n, window, True, False)
    f = int_freq(n).astype(float)
    th = [2 * math.pi * f[:, None, None] / n, 2 * math.pi * f[None, :, None] / n, 2 * math.pi * f[None, None, :] / n]
    half = np.cos(th[0] / 2) * np.cos(th[1] / 2) * np.cos(th[2] / 2)
    a = np.ones_like(half) if window == CIC else (0.75 + 0.25 * np.cos(th[0])) * (0.75 + 0.25 * np.cos(th[1])) * (0.75 + 0.25 * np.cos(th[2]))
    ph = np.exp(-1j * (th[0] * p[0] + th[1] * p[1] + th[2] * p[2]))
    ref = 0.5 * (a + half) * ph
    mask = nyquist_mask(n)
    assert np.max(np.abs(c[mask] - ref[mask])) < 1e-14
    assert np.all(c[~mask] == 0)


@pytest.mark.parametrize("window,p", [(CIC, 2), (TSC, 3)])
def test_jing_alias_sums(window, p):
    """sum_m sinc^(2p)(x + pi m) over images equals the closed form squared in compensation_1d
    (non-interlaced) for CIC and TSC."""
    n = 16
    f = int_freq(n).astype(float)
    x = math.pi * f / n
    m = np.arange(-3000, 3001)[:, None]
    arg = x[None, :] + math.pi * m
    with np.errstate(invalid="ignore", divide="ignore"):
        s = np.where(arg == 0, 1.0, np.sin(arg) / arg)
    brute = np.sum(s ** (2 * p), axis=0)
    assert np.max(np.abs(compensation_1d(n, window, False) ** 2 - brute)) < 1e-10
    # interlaced form: plain sinc^p
    with np.errstate(invalid="ignore", divide="ignore"):
        sinc = np.where(f == 0, 1.0, np.sin(x) / np.where(f == 0, 1.0, x))
    assert np.max(np.abs(compensation_1d(n, window, True) - sinc ** window)) < 1e-15
    assert np.all(compensation_1d(n, NGP, False) == 1.0)


@pytest.mark.parametrize("window", [NGP, CIC, TSC])
def test_paint_at_matches_tap_painting(window):
    """The kernel-definition evaluation at chosen nodes equals the tap painter there,
    including nodes reached through the periodic wrap."""
    rng = np.random.default_rng(11 + window)
    n = 12
    u = rng.random((300, 3)) * n
    u[:20] = rng.random((20, 3)) * 1.2 - 0.6          # straddling the wrap at 0
    u[20:25] = np.floor(u[20:25]) + 0.5                # exactly on a cell edge
    w = rng.normal(size=300)
    full = paint(u, w, n, window)
    cells = np.array([[i, j, k] for i in (0, 1, 5, 11) for j in (0, 6, 11) for k in (0, 3, 11)])
    got = paint_at(u, w, n, window, cells)
    ref = full[cells[:, 0], cells[:, 1], cells[:, 2]]
    assert np.allclose(got, ref, rtol=0, atol=1e-13 * np.sum(np.abs(w)))


def test_window_kernels_closed_form():
    d = np.array([-1.6, -1.5, -1.0, -0.5, -0.25, 0.0, 0.25, 0.5, 1.0, 1.5])
    assert np.array_equal(window_1d(d, NGP), [0, 0, 0, 1, 1, 1, 1, 0, 0, 0])
    assert np.allclose(window_1d(d, CIC), [0, 0, 0, 0.5, 0.75, 1, 0.75, 0.5, 0, 0])
    assert np.allclose(window_1d(d, TSC), [0, 0, 0.125, 0.5, 0.6875, 0.75, 0.6875, 0.5, 0.125, 0])
