"""Deterministic mode (pkm_params.deterministic): painting sums fixed-point integers (one
scale shared by all tiles) in LDS and in 64-bit accumulators, and the post-pass keeps one
histogram per wavefront, so an estimate repeats bit for bit.

Catalogs are clustered (a third of the objects in a ball of a few cells) so that many taps of
one tile, and tiles' halos, land on the same nodes: the case where floating-point atomics
make the default mode's sums depend on scheduling.  Every deterministic result is also
compared with the FP64 oracle to the form's tolerance, and with the default mode."""
from __future__ import annotations

import math

import numpy as np
import pytest

from tests.parity_util import assert_pole_parity, oracle_params, small_catalogs

pytestmark = pytest.mark.gpu

OBS = (30.0, -40.0, -700.0)
L = 300.0


def _clustered(nd, nr, seed):
    from synth import Catalog
    d, r = small_catalogs(nd, nr, L, seed=seed)
    rng = np.random.default_rng(seed + 1)
    k = nd // 3
    pos = d.pos.copy()
    pos[:k] = 12.0 + rng.normal(scale=6.0, size=(k, 3))  # a few cells of a 64^3 mesh
    pos = np.clip(pos, -0.5 * L, 0.5 * L - 1e-9)
    return Catalog(pos, d.w, d.nbar), r


def _edges(n):
    return np.arange(0.0, math.pi * n / L, 0.04)


@pytest.mark.parametrize("prec", [1, 0])
def test_repeat_paint_is_bitwise_equal(gpu, prec):
    from paper_1704_02357_amd import Plan
    n = 64
    d, r = _clustered(60_000, 240_000, seed=11 + prec)
    d2, r2 = _clustered(30_000, 90_000, seed=91 + prec)
    kw = dict(observer=OBS, window=3, interlaced=True, compensated=True, precision=prec, ell_max_hint=8)
    p = Plan(n, L, deterministic=True, **kw)
    q = Plan(n, L, deterministic=True, **kw)
    runs = []
    for plan, cats in ((p, (d, r)), (p, (d2, r2)), (p, (d, r)), (q, (d, r))):
        plan.paint(*cats)
        if cats[0] is d:
            runs.append((plan.read_buffer(0).copy(), plan.read_buffer(1).copy(), plan.read_buffer(2).copy(),
                         plan.compute_multipoles(8, _edges(n)), plan.compute_multipoles(8, _edges(n))))
    print(f"[case] deterministic repeat prec={prec}", flush=True)
    a = runs[0]
    for b in runs[1:]:
        for i in range(3):
            assert np.array_equal(a[i], b[i]), f"buffer {i} differs"
        for res in (b[3], b[4]):
            for key in ("poles", "k_mean", "n_modes"):
                assert np.array_equal(np.asarray(a[3][key]), np.asarray(res[key]), equal_nan=True), key
            for key in ("alpha", "norm_I", "shot_noise"):
                assert a[3][key] == res[key], key
    from oracle.estimator import multipoles
    ref = multipoles(d, r, oracle_params(n, L, OBS, 3, True, True), 8, _edges(n))
    assert_pole_parity(a[3], ref, prec, f"deterministic 64^3 prec={prec} vs oracle")
    plain = Plan(n, L, **kw)
    plain.paint(d, r)
    assert_pole_parity(plain.compute_multipoles(8, _edges(n)), ref, prec, f"default mode 64^3 prec={prec} vs oracle")
    plain.close()
    p.close()
    q.close()


def test_batch_and_server_equal_alone_bitwise(gpu):
    """A deterministic plan in a batch (direct issue and graph replays) and a deterministic
    served request give the synchronous result bit for bit."""
    import torch
    from paper_1704_02357_amd import Batch, Plan, Server
    n, prec = 48, 1
    d, r = _clustered(20_000, 80_000, seed=5)
    kw = dict(observer=OBS, window=3, interlaced=True, compensated=True, precision=prec, ell_max_hint=4,
              deterministic=True)
    alone = Plan(n, L, **kw)
    alone.paint(d, r)
    ref = alone.compute_multipoles(4, _edges(n))
    alone.close()
    dev = lambda c: (torch.tensor(c.pos, device="cuda"), torch.tensor(c.w, device="cuda"),
                     torch.tensor(c.nbar, device="cuda"))
    p = Plan(n, L, stream=torch.cuda.Stream(), **kw)
    p.prepare(4, _edges(n), len(d.pos) + len(r.pos))
    b = Batch()
    b.add(p, dev(d), dev(r))
    for use_graph in (False, True, True):
        b.run(use_graph=use_graph)
        got = b.result(0)
        assert np.array_equal(got["poles"], ref["poles"], equal_nan=True), f"batch graph={use_graph}"
    b.close()
    p.close()
    sv = Server(max_inflight=2)
    t = sv.submit(n, L, 4, _edges(n), d, r, **kw)
    got = sv.wait(t)
    sv.close()
    assert np.array_equal(got["poles"], ref["poles"], equal_nan=True)
