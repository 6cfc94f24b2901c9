"""Pins of the oracle's odd multipoles R_l (reading: the shell average of eq. Pell-ours is
purely imaginary for odd l, P_l = i R_l, R_l = (2l+1)/(I N_i) sum Im[C conj A_l] with the
transforms' exponent exp(-i k.x); eq. Pell-yama gives -i R_l for odd l).

* O3 (FFT, spherical harmonics) against O1 (literal Legendre-weighted DFT), every l <= 16;
* O3 against O2 (galaxy-direct sums) exactly for particles on mesh nodes;
* the paper's complex shell averages written out literally (each F evaluated as its own
  direct sum at the wave vector it needs, exponent +i k.r as in eq. Fell): for odd l, real
  part zero and imaginary part R_l for eq. Pell-ours and -R_l for eq. Pell-yama; for even l,
  both real, P_l + S delta_l0;
* inverting the catalog and the observer through the box centre keeps every multipole, and
  an observer far above the box gives the same odd multipoles as one far below (to second
  order in the opening angle: the odd signal is the transverse spread of the lines of sight);
* with a receding observer the odd multipoles vanish like the opening angle L/D (they are a
  wide-angle effect) while the even ones tend to their plane-parallel values.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle.direct import brute_force_multipoles, pell_complex_literal, shell_modes, yamamoto_at_modes
from oracle.estimator import all_multipoles, default_params, k_thresholds
from synth import Catalog


def _cat(n, L, seed, npart=300, origin=None):
    rng = np.random.default_rng(seed)
    o = -0.5 * L if origin is None else origin
    return Catalog(o + rng.random((npart, 3)) * L, rng.uniform(0.5, 1.5, npart), np.full(npart, npart / L ** 3))


def _on_node(n, L, npart, seed):
    rng = np.random.default_rng(seed)
    pos = -0.5 * L + rng.integers(0, n, size=(npart, 3)) * (L / n)
    return Catalog(pos, rng.uniform(0.5, 1.5, npart), np.full(npart, npart / L ** 3))


def _scale(res):
    return np.abs(res["poles"][0] + res["shot_noise"])[None, :]


def test_odd_fft_oracle_equals_brute_force():
    n, L = 12, 150.0
    d, r = _cat(n, L, 1, 200), _cat(n, L, 2, 800)
    p = default_params(n, L, observer=(20.0, -30.0, -260.0), window=3, interlaced=True, compensated=True)
    edges = np.linspace(0.02, math.pi * n / L, 6)
    res = all_multipoles(d, r, p, 16, edges)
    bf, cnt = brute_force_multipoles(d, r, p, list(range(17)), edges)
    assert np.array_equal(cnt.astype(np.int64), res["n_modes"])
    err = np.max(np.abs(res["poles"] - bf) / _scale(res))
    assert err < 1e-12, err
    # the odd rows are not trivially zero
    assert np.min(np.max(np.abs(res["poles"][1::2]), axis=1) / np.max(_scale(res))) > 1e-6


def test_odd_fft_oracle_equals_direct_sums_on_nodes():
    n, L = 16, 200.0
    d = _on_node(n, L, 250, 3)
    p = default_params(n, L, observer=(11.0, 5.0, -350.0), window=1, interlaced=False, compensated=False)
    edges = np.linspace(0.02, math.pi * n / L, 7)
    res = all_multipoles(d, None, p, 16, edges)
    thr = k_thresholds(edges, L)
    modes, b = shell_modes(n, thr, range(thr.size - 1))
    o2, cnt, _ = yamamoto_at_modes(d, None, p, list(range(17)), modes, b, thr.size - 1)
    assert np.array_equal(cnt.astype(np.int64), res["n_modes"])
    assert np.max(np.abs(res["poles"] - o2) / _scale(res)) < 1e-12


def test_literal_complex_average_fixes_the_reading():
    n, L = 16, 200.0
    d = _on_node(n, L, 250, 4)
    p = default_params(n, L, observer=(-17.0, 23.0, -300.0), window=1, interlaced=False, compensated=False)
    edges = np.linspace(0.02, math.pi * n / L, 6)
    res = all_multipoles(d, None, p, 9, edges)
    thr = k_thresholds(edges, L)
    modes, b = shell_modes(n, thr, range(thr.size - 1))
    sc = _scale(res)[0]
    for ell in range(10):
        for form, sign in (("ours", 1.0), ("yama", -1.0)):
            z = pell_complex_literal(d, None, p, ell, modes, b, thr.size - 1, form=form)
            if ell % 2:
                assert np.max(np.abs(z.real) / sc) < 1e-12
                assert np.max(np.abs(z.imag - sign * res["poles"][ell]) / sc) < 1e-12
                assert np.max(np.abs(z.imag) / sc) > 1e-5       # a real signal, with a fixed sign
            else:
                shot = res["shot_noise"] if ell == 0 else 0.0
                assert np.max(np.abs(z.real - res["poles"][ell] - shot) / sc) < 1e-12
                assert np.max(np.abs(z.imag) / sc) < 1e-12


def test_inversion_keeps_every_multipole():
    """Inverting the catalog and the observer together (an orthogonal map of the whole
    configuration) leaves every multipole, odd ones included, unchanged.  Node c maps to node
    -c (mod N), except that the plane c_a = 0 sits at -L/2 and its image at +L/2: the catalogs
    stay in the central 60% of the box and the field is not compensated (no ringing), so
    nothing is painted on that plane."""
    n, L = 16, 200.0
    central = lambda c: Catalog(0.6 * c.pos, c.w, c.nbar)
    d, r = central(_cat(n, L, 5, 300)), central(_cat(n, L, 6, 1500))
    obs = np.array([23.0, -41.0, -330.0])
    p = default_params(n, L, observer=tuple(obs), window=2, interlaced=False, compensated=False)
    pi = default_params(n, L, observer=tuple(-obs), window=2, interlaced=False, compensated=False)
    edges = np.linspace(0.02, math.pi * n / L, 7)
    inv = lambda c: Catalog(-c.pos, c.w, c.nbar)
    a = all_multipoles(d, r, p, 7, edges)
    b = all_multipoles(inv(d), inv(r), pi, 7, edges)
    assert np.max(np.abs(b["poles"] - a["poles"]) / _scale(a)) < 1e-10
    assert np.max(np.abs(a["poles"][1::2]) / _scale(a)) > 1e-5


def test_odd_multipoles_keep_their_sign_across_the_box():
    """An observer far below the box (line of sight zhat + x_perp/D) and one as far above it
    (-zhat + x_perp/D): for odd l, L_l(-mu + e) = -L_l(mu - e), so the plane-parallel part
    flips (and vanishes in the shell average anyway) while the first-order part
    L_l'(mu) khat . x_perp / D, which carries the whole odd signal, keeps its sign.  Both
    observers give the same odd multipoles to O((L/D)^2); for even l the first-order part
    flips instead, so the even multipoles agree only to O(L/D)."""
    n, L = 16, 200.0
    d = _cat(n, L, 8, 400)
    edges = np.linspace(0.02, math.pi * n / L, 6)
    D = 1000.0 * L
    lo = all_multipoles(d, None, default_params(n, L, observer=(0.0, 0.0, -D), window=2, interlaced=False,
                                                compensated=True), 5, edges)
    hi = all_multipoles(d, None, default_params(n, L, observer=(0.0, 0.0, D), window=2, interlaced=False,
                                                compensated=True), 5, edges)
    sc = _scale(lo)
    odd = np.max(np.abs(lo["poles"][1::2]) / sc)
    assert np.max(np.abs(hi["poles"][1::2] - lo["poles"][1::2]) / sc) < 1e-2 * odd
    even = np.max(np.abs(hi["poles"][0::2] - lo["poles"][0::2]) / sc)
    assert even < 10.0 * L / D and even > 10.0 * np.max(np.abs(hi["poles"][1::2] - lo["poles"][1::2]) / sc)


def test_odd_multipoles_vanish_for_a_distant_observer():
    n, L = 16, 200.0
    d = _cat(n, L, 7, 400)
    edges = np.linspace(0.02, math.pi * n / L, 6)
    odd = []
    for dist in (10.0, 1000.0, 1e9):
        p = default_params(n, L, observer=(0.0, 0.0, -dist * L), window=2, interlaced=False, compensated=True)
        res = all_multipoles(d, None, p, 5, edges)
        odd.append(np.max(np.abs(res["poles"][1::2]) / _scale(res)))
    ratio = odd[1] / odd[0]
    assert 0.002 < ratio < 0.05, ratio      # ~ L/D: a factor 100 in distance
    assert odd[2] < 1e-8
