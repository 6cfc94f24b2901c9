"""Pins of the oracle's fixed line-of-sight (k, mu) cells against exact integer arithmetic.

mu = |khat . lhat| decides the mu bin of every mode (Sec. 2.2 wedges, plane-parallel
limit of Sec. 1).  Here every decision is redone without floating point: for a rational
unit vector lhat = v/q (integer v, |v| = q) and a rational edge e = a/b,

    mu >= e   <=>   b^2 (n . v)^2 >= a^2 q^2 |n|^2,

and the k bin is T_i <= |n|^2 < T_{i+1} for integer thresholds.  Bins are left-closed and
mu = 1 belongs to the last bin.  The reference is then compared mode by mode with
``oracle.global_los.mu_bins(mode_mu(...))`` and cell by cell with the counts of
``oracle.global_los.pkmu``.  Each test also checks that the plausible mistakes (a swapped or
misplaced line-of-sight component, right-closed bins) change the exact reference, so a
mistake of that kind in the oracle would fail it.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from oracle.estimator import default_params
from oracle.global_los import mode_mu, mu_bins, pkmu
from oracle.mesh import int_freq, nyquist_mask
from synth import Catalog

N = 16


def _modes(n):
    f = int_freq(n)
    fx, fy, fz = np.meshgrid(f, f, f, indexing="ij")
    return fx, fy, fz


def exact_mu_bins(n, v, q, edges, right_closed=False):
    """mu bin of every full-grid mode from integers only; -1 for n = 0.

    v: integer 3-vector with |v| = q; edges: Fractions 0 = e_0 < ... < e_m = 1.
    """
    fx, fy, fz = _modes(n)
    dot = fx * v[0] + fy * v[1] + fz * v[2]
    n2 = fx * fx + fy * fy + fz * fz
    lhs = dot * dot  # (n . v)^2, compared against e^2 q^2 |n|^2
    nm = len(edges) - 1
    out = np.full(fx.shape, -1, dtype=np.int64)
    it = np.nditer(lhs, flags=["multi_index"])
    for d2 in it:
        idx = it.multi_index
        m2 = int(n2[idx])
        if m2 == 0:
            continue
        d2 = int(d2)
        j = -1
        for k in range(nm):
            a, b = edges[k].numerator, edges[k].denominator
            a1, b1 = edges[k + 1].numerator, edges[k + 1].denominator
            if right_closed:
                above_lo = b * b * d2 > a * a * q * q * m2
                below_hi = b1 * b1 * d2 <= a1 * a1 * q * q * m2
            else:
                above_lo = b * b * d2 >= a * a * q * q * m2
                below_hi = b1 * b1 * d2 < a1 * a1 * q * q * m2
            if above_lo and below_hi:
                j = k
                break
        if j < 0 and b1 * b1 * d2 >= a1 * a1 * q * q * m2:  # mu = 1 (or above the last edge)
            j = nm - 1
        out[idx] = j
    return out


def exact_k_bins(n, thr):
    fx, fy, fz = _modes(n)
    n2 = fx * fx + fy * fy + fz * fz
    kb = np.full(n2.shape, -1, dtype=np.int64)
    for i in range(len(thr) - 1):
        kb[(n2 >= thr[i]) & (n2 < thr[i + 1])] = i
    kb[n2 == 0] = -1
    kb[~nyquist_mask(n)] = -1
    return kb


def _ties(n, v, q, edges):
    fx, fy, fz = _modes(n)
    d2 = (fx * v[0] + fy * v[1] + fz * v[2]) ** 2
    m2 = fx * fx + fy * fy + fz * fz
    t = 0
    for e in edges[1:-1]:
        t += int(np.sum((m2 > 0) & (e.denominator ** 2 * d2 == e.numerator ** 2 * q * q * m2)))
    return t


# lhat = zhat: direction cosines exact in FP64, so ties with rational edges (mu = 1/3 at
# (2, 2, 1), 3/5 at (4, 0, 3), 2/3 at (1, 2, 2), 4/5 at (0, 3, 4)) are decided exactly
Z_EDGES = [Fraction(0), Fraction(1, 3), Fraction(3, 5), Fraction(2, 3), Fraction(4, 5), Fraction(1)]
# lhat = (1, 2, 2)/3: components inexact in FP64, so the edges are chosen with no exact tie
# on the grid (checked below) and the FP64 decision is unambiguous
D_EDGES = [Fraction(0), Fraction(23, 100), Fraction(41, 100), Fraction(57, 100), Fraction(78, 100),
           Fraction(93, 100), Fraction(1)]


def test_exact_reference_is_sensitive():
    """The integer reference separates the mistakes the pins must catch."""
    ref_z = exact_mu_bins(N, (0, 0, 1), 1, Z_EDGES)
    assert _ties(N, (0, 0, 1), 1, Z_EDGES) > 0
    # right-closed bins move every tie mode
    assert not np.array_equal(ref_z, exact_mu_bins(N, (0, 0, 1), 1, Z_EDGES, right_closed=True))
    # a line of sight along x instead of z
    assert not np.array_equal(ref_z, exact_mu_bins(N, (1, 0, 0), 1, Z_EDGES))
    ref_d = exact_mu_bins(N, (1, 2, 2), 3, D_EDGES)
    assert _ties(N, (1, 2, 2), 3, D_EDGES) == 0
    for wrong in ((2, 1, 2), (2, 2, 1), (2, 2, 2), (-1, 2, 2)):
        qq = math.isqrt(sum(c * c for c in wrong))
        assert not np.array_equal(ref_d, exact_mu_bins(N, wrong, qq if qq * qq == sum(c * c for c in wrong) else 3,
                                                       D_EDGES))
    # mu = 1 modes (n parallel to lhat) sit in the last bin
    fx, fy, fz = _modes(N)
    par = (fx == 0) & (fy == 0) & (fz != 0)
    assert np.all(ref_z[par] == len(Z_EDGES) - 2)
    par_d = (fx != 0) & (fy == 2 * fx) & (fz == 2 * fx)
    assert par_d.any() and np.all(ref_d[par_d] == len(D_EDGES) - 2)


def _nonzero():
    fx, fy, fz = _modes(N)
    return (fx * fx + fy * fy + fz * fz) > 0  # n = 0 has no direction and is in no k bin


def test_mu_bins_match_exact_integers_zhat():
    got = mu_bins(mode_mu(N, (0.0, 0.0, 1.0)), [float(e) for e in Z_EDGES])
    ref = exact_mu_bins(N, (0, 0, 1), 1, Z_EDGES)
    nz = _nonzero()
    assert np.array_equal(got[nz], ref[nz])


def test_mu_bins_match_exact_integers_oblique():
    got = mu_bins(mode_mu(N, (1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0)), [float(e) for e in D_EDGES])
    ref = exact_mu_bins(N, (1, 2, 2), 3, D_EDGES)
    nz = _nonzero()
    assert np.array_equal(got[nz], ref[nz])


def test_pkmu_cell_counts_match_exact_integers():
    """Per-(k, mu) mode counts of the oracle's P(k, mu) against the integer reference."""
    L = 300.0
    rng = np.random.default_rng(5)
    pos = -L / 2 + rng.random((400, 3)) * L
    cat = Catalog(pos, np.ones(400), np.full(400, 400 / L ** 3))
    thr = np.array([1, 5, 11, 20, 33, 49], dtype=np.int64)
    kf = 2.0 * math.pi / L
    # k edges whose thresholds ceil((e L / 2 pi)^2) are exactly `thr` (half a unit below)
    k_edges = kf * np.sqrt(thr - 0.5)
    kb = exact_k_bins(N, thr)
    p = default_params(N, L, window=2, interlaced=False, compensated=False)
    for v, q, edges, los in (((0, 0, 1), 1, Z_EDGES, (0.0, 0.0, 1.0)),
                             ((1, 2, 2), 3, D_EDGES, (1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0))):
        mb = exact_mu_bins(N, v, q, edges)
        nk, nm = len(thr) - 1, len(edges) - 1
        ref = np.zeros((nk, nm), dtype=np.int64)
        ok = (kb >= 0) & (mb >= 0)
        np.add.at(ref, (kb[ok], mb[ok]), 1)
        _, cnt = pkmu(cat, None, p, k_edges, [float(e) for e in edges], los)
        assert np.array_equal(cnt, ref), (v, cnt, ref)
        assert np.all(ref.sum(axis=0) > 0) and np.all(ref.sum(axis=1) > 0)  # no bin passes vacuously
