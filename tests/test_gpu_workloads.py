"""GPU parity on the full-size survey workloads, in the configuration bench.py times.

* 64^3, L = 1000 Mpc/h, CIC, l <= 4 (3e4 lognormal galaxies, 10x randoms): the oracle runs
  live, both precision forms.
* 512^3, L = 2500 Mpc/h, TSC + interlacing + compensation, l <= 4 (1e6 galaxies, 2e7
  randoms): P_l(k) against the oracle's values stored by tests/golden/make_workload_golden.py
  (an oracle-only script; the catalog digest is checked first), and the painted meshes at
  sampled nodes against the oracle's kernel-definition painter.
* 1024^3, L = 3000 Mpc/h, TSC + interlacing, l <= 16 (4e6 galaxies, 4e7 randoms): painted
  meshes at sampled nodes and the per-bin mode counts; the multipoles themselves are checked
  for finiteness and FP32/FP64 agreement only (no oracle value exists at this size).
"""
from __future__ import annotations

import math
import os

import numpy as np
import pytest

from tests.parity_util import TOL, assert_pole_parity, oracle_params

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN_512 = os.path.join(HERE, "golden", "workload_512_l4_poles.txt")
OBS = (0.0, 0.0, -1500.0)


def _edges(n, L, dk=0.01):
    kn = math.pi * n / L
    return np.arange(int(math.floor(kn / dk)) + 1, dtype=np.float64) * dk


def _plan(n, L, prec, window, interlaced, compensated, lmax, max_group=0):
    from paper_1704_02357_amd import Plan
    return Plan(n, L, observer=OBS, window=window, interlaced=interlaced, compensated=compensated,
                precision=prec, ell_max_hint=lmax, max_group=max_group)


def load_golden(path):
    meta, rows = {}, []
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                parts = line[1:].split()
                if parts and parts[0] in ("alpha", "norm_I", "shot_noise"):
                    meta[parts[0]] = float(parts[1])
                if parts and parts[0] == "catalog:":
                    meta["digest"] = parts[parts.index("digest") + 1]
                continue
            rows.append(line.split())
    t = np.array([[float(v) for v in r] for r in rows])
    return {"edges": np.append(t[:, 0], t[-1, 1]), "n_modes": t[:, 2].astype(np.int64), "k_mean": t[:, 3],
            "poles": t[:, 4:].T.copy(), "alpha": meta["alpha"], "norm_I": meta["norm_I"],
            "shot_noise": meta["shot_noise"], "digest": meta["digest"]}


# ---------------------------------------------------------------------------------------------
# sampled painted nodes (any size)
# ---------------------------------------------------------------------------------------------
def sampled_nodes(data, rand, n, L, origin, rng, k_occupied=120, k_random=40):
    """Nodes where the catalog has particles, random nodes, and nodes on the box faces."""
    from oracle.mesh import mesh_coords
    u = mesh_coords(rand.pos[:: max(1, len(rand.pos) // 200000)], L, origin, n)
    occ = np.floor(u[rng.integers(0, len(u), k_occupied)]).astype(np.int64) % n
    rnd = rng.integers(0, n, (k_random, 3))
    faces = np.array([[0, 0, 0], [n - 1, n - 1, n - 1], [0, n // 2, n - 1], [n - 1, 0, n // 3]])
    return np.concatenate([occ, rnd, faces])


def expected_at_nodes(data, rand, n, L, origin, window, nodes, shift):
    """Oracle painting of D = sum_d w W - alpha sum_r w W at the nodes (and sum of |terms|)."""
    from oracle.catalog import catalog_scalars
    from oracle.mesh import mesh_coords, paint_at
    alpha = catalog_scalars(data, rand, L)["alpha"]
    reach = 2
    # ids of the cells within `reach` of a sampled node on every axis
    off = np.arange(-reach, reach + 1)
    nb = (nodes[:, None, None, None, :] + np.stack(np.meshgrid(off, off, off, indexing="ij"), -1)[None]) % n
    ids = np.unique(((nb[..., 0] * n + nb[..., 1]) * n + nb[..., 2]).ravel())
    val = np.zeros(len(nodes))
    mag = np.zeros(len(nodes))
    for cat, sign in ((data, 1.0), (rand, -alpha)):
        u = mesh_coords(cat.pos, L, origin, n) + (0.5 if shift else 0.0)
        c = np.floor(u).astype(np.int64) % n
        keep = np.isin((c[:, 0] * n + c[:, 1]) * n + c[:, 2], ids)
        w = sign * (np.ones(len(u)) if cat.w is None else cat.w)
        val += paint_at(u[keep], w[keep], n, window, nodes)
        mag += paint_at(u[keep], np.abs(w[keep]), n, window, nodes)
    return val, mag


def check_sampled_paint(plan, data, rand, n, L, window, interlaced, prec, seed):
    rng = np.random.default_rng(seed)
    origin = (-0.5 * L,) * 3
    nodes = sampled_nodes(data, rand, n, L, origin, rng)
    tol = 1e-12 if prec else 2e-6
    for which, shift in ((0, False), (1, True)) if interlaced else ((0, False),):
        g = plan.read_buffer(which)
        got = g[nodes[:, 0], nodes[:, 1], nodes[:, 2]].astype(np.float64)
        del g
        exp, mag = expected_at_nodes(data, rand, n, L, origin, window, nodes, shift)
        err = np.abs(got - exp) / np.maximum(mag, 1e-300)
        print(f"[paint] n={n} prec={prec} mesh={which} nodes={len(nodes)} nonzero={int(np.sum(mag > 0))} "
              f"max_rel_err={err.max():.3e}", flush=True)
        assert np.sum(mag > 0) >= len(nodes) // 2
        assert err.max() <= tol


# ---------------------------------------------------------------------------------------------
# 64^3, l <= 4: live oracle
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("prec", [1, 0])
def test_workload_64_l4_live_oracle(gpu, prec):
    from oracle.estimator import multipoles
    from synth import config_c1
    data, rand, info = config_c1()
    n, L = 64, 1000.0
    edges = _edges(n, L)
    print(f"[case] 64^3 l<=4 prec={prec} n_data={info['n_data']} n_rand={info['n_rand']}", flush=True)
    plan = _plan(n, L, prec, 2, False, True, 4)
    plan.paint(data, rand)
    got = plan.compute_multipoles(4, edges)
    ref = multipoles(data, rand, oracle_params(n, L, OBS, 2, False, True), 4, edges, workers=8)
    assert_pole_parity(got, ref, prec, "64^3 CIC l<=4")
    plan.close()


# ---------------------------------------------------------------------------------------------
# 512^3, l <= 4: the timed workload
# ---------------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def workload_512():
    from synth import catalog_digest, config_c2
    data, rand, info = config_c2()
    return data, rand, info, catalog_digest(data, rand)


@pytest.mark.parametrize("prec", [0, 1])
def test_workload_512_l4_vs_stored_oracle(gpu, workload_512, prec):
    data, rand, info, digest = workload_512
    gold = load_golden(GOLDEN_512)
    assert digest == gold["digest"], "the seeded catalog differs from the one the stored oracle values belong to"
    n, L = 512, 2500.0
    edges = _edges(n, L)
    assert np.array_equal(edges, gold["edges"])
    print(f"[case] 512^3 l<=4 prec={prec}", flush=True)
    plan = _plan(n, L, prec, 3, True, True, 4)
    plan.paint(data, rand)
    got = plan.compute_multipoles(4, edges)
    assert got["n_transforms"] == 17
    assert_pole_parity(got, gold, prec, "512^3 TSC interlaced l<=4")
    check_sampled_paint(plan, data, rand, n, L, 3, True, prec, seed=512 + prec)
    plan.close()


# ---------------------------------------------------------------------------------------------
# 1024^3, l <= 16: sampled nodes, mode counts, FP32 against FP64
# ---------------------------------------------------------------------------------------------
def test_workload_1024_l16(gpu):
    from oracle.estimator import k_thresholds
    from synth import config_c3
    data, rand, info = config_c3()
    n, L = 1024, 3000.0
    edges = _edges(n, L)
    res = {}
    for prec in (0, 1):
        print(f"[case] 1024^3 l<=16 prec={prec}", flush=True)
        # 24 weighted fields resident at a time (8.6 GB each at FP64): 153 fields in 7 groups
        plan = _plan(n, L, prec, 3, True, True, 16, max_group=24)
        plan.paint(data, rand)
        if prec == 0:
            check_sampled_paint(plan, data, rand, n, L, 3, True, prec, seed=1024)
        res[prec] = plan.compute_multipoles(16, edges)
        assert res[prec]["n_transforms"] == 152 + 3   # 153 harmonic fields less l = 0, plus 2 forward + 1 inverse
        plan.close()
    # mode counts: integer squared radii against the oracle's thresholds, counted per kz plane
    thr = k_thresholds(edges, L)
    f = np.fft.fftfreq(n, 1.0 / n).astype(np.int64)
    f[n // 2] = 0
    fx2 = f[:, None] ** 2 + f[None, :] ** 2
    ok_xy = np.ones((n, n), dtype=bool)
    ok_xy[n // 2, :] = ok_xy[:, n // 2] = False
    counts = np.zeros(len(edges) - 1, dtype=np.int64)
    for kz in range(n // 2):
        n2 = fx2[ok_xy] + kz * kz
        b = np.searchsorted(thr, n2, side="right") - 1
        good = (b >= 0) & (b < len(edges) - 1) & (n2 > 0)
        counts += (1 if kz == 0 else 2) * np.bincount(b[good], minlength=len(edges) - 1)
    assert np.array_equal(res[0]["n_modes"], counts)
    assert np.array_equal(res[1]["n_modes"], counts)
    p32, p64 = res[0]["poles"], res[1]["poles"]
    ok = np.isfinite(p64)
    assert np.array_equal(ok, np.isfinite(p32))
    scale = np.maximum(np.abs(p64), np.abs(p64[0] + res[1]["shot_noise"])[None, :])
    err = np.max(np.abs(p32 - p64)[ok] / scale[ok])
    print(f"[parity] 1024^3 l<=16 fp32 vs fp64 scaled_err={err:.3e}", flush=True)
    assert err <= TOL[0]
