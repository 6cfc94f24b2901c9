"""GPU tests of the asynchronous estimate, the batch runtime (uneven mock sizes, HIP graph
capture and replay) and the serving loop (mixed requests admitted while others run).

Every batched or served result is compared with the FP64 oracle and with the same estimate
run alone through the synchronous calls, each to the precision form's tolerance."""
from __future__ import annotations

import math

import numpy as np
import pytest

from tests.parity_util import small_catalogs

pytestmark = pytest.mark.gpu

OBS = (30.0, -40.0, -700.0)
L = 300.0


def _edges(n):
    return np.arange(0.0, math.pi * n / L, 0.04)


def _scaled_err(a, b):
    pa, pb = np.asarray(a["poles"]), np.asarray(b["poles"])
    scale = np.maximum(np.abs(pb), np.abs(pb[0] + b["shot_noise"])[None, :])
    ok = np.isfinite(pb)
    assert np.array_equal(ok, np.isfinite(pa))
    return float(np.max(np.abs(pa - pb)[ok] / scale[ok])) if ok.any() else 0.0


# painting adds tile flushes with atomics, so two runs agree to rounding only
RUN_TOL = {0: 2e-6, 1: 1e-12}


def _same(a, b, prec, label):
    assert np.array_equal(a["n_modes"], b["n_modes"]), label
    for k in ("alpha", "norm_I", "shot_noise"):
        assert abs(a[k] - b[k]) <= 1e-12 * abs(b[k]), (label, k)
    err = _scaled_err(a, b)
    print(f"[same] {label} scaled_err={err:.2e}", flush=True)
    assert err <= RUN_TOL[prec], (label, err)


def _plan(n, prec, lmax=4, stream=None, **kw):
    from paper_1704_02357_amd import Plan
    return Plan(n, L, observer=OBS, window=3, interlaced=True, compensated=True, precision=prec,
                ell_max_hint=lmax, stream=stream, **kw)


def _alone(n, prec, lmax, d, r, **kw):
    p = _plan(n, prec, lmax, **kw)
    p.paint(d, r)
    out = p.compute_multipoles(lmax, _edges(n))
    p.close()
    return out


def _oracle(n, lmax, d, r):
    from oracle.estimator import multipoles
    from tests.parity_util import oracle_params
    return multipoles(d, r, oracle_params(n, L, OBS, 3, True, True), lmax, _edges(n))


def _dev(cat):
    import torch
    if cat is None:
        return None
    f = lambda a: None if a is None else torch.tensor(a, dtype=torch.float64, device="cuda")
    return (f(cat.pos), f(cat.w), f(cat.nbar))


@pytest.mark.parametrize("prec", [0, 1])
def test_async_estimate_matches_sync(gpu, prec):
    import torch
    from paper_1704_02357_amd import PkmError
    n, lmax = 48, 4
    d, r = small_catalogs(3000, 20000, L, seed=71)
    ref = _alone(n, prec, lmax, d, r)
    s = torch.cuda.Stream()
    p = _plan(n, prec, lmax, stream=s)
    dd, rr = _dev(d), _dev(r)
    with pytest.raises(PkmError):          # not prepared
        p.enqueue(dd, rr)
    p.prepare(lmax, _edges(n), 30000)
    with pytest.raises(PkmError):          # host catalogs are refused
        p.enqueue(d, r)
    p.enqueue(dd, rr)
    with pytest.raises(PkmError):          # one estimate at a time
        p.enqueue(dd, rr)
    with pytest.raises(PkmError):          # the plan's buffers are in use
        p.paint(d, r)
    while not p.query():
        pass
    got = p.finish()
    _same(got, ref, prec, f"async prec={prec}")
    # the plan now holds the painted field: a synchronous compute agrees
    again = p.compute_multipoles(lmax, _edges(n))
    _same(again, ref, prec, f"after finish prec={prec}")
    # a synchronous request with other settings replaces the prepared one: enqueue refuses
    # (its result slot was sized for the prepared request) until the plan is prepared again
    from paper_1704_02357_amd import CARTESIAN
    for other in (dict(ell_max=8, k_edges=_edges(n)), dict(ell_max=lmax, k_edges=_edges(n)[:-3]),
                  dict(ell_max=lmax, k_edges=_edges(n), basis=CARTESIAN)):
        p.compute_multipoles(**other)
        with pytest.raises(PkmError) as e:
            p.enqueue(dd, rr)
        assert e.value.status == 2
    p.prepare(lmax, _edges(n), 30000)
    p.enqueue(dd, rr)
    _same(p.finish(), ref, prec, f"re-prepared prec={prec}")
    p.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_estimates_in_flight_on_two_plans(gpu, prec):
    """The benchmark's headline loop: estimate i on plan i mod 2, each plan on its own stream, a
    plan's previous estimate finished before its next is enqueued, so two estimates (of two
    catalogs here) overlap on the device.  Every result equals its catalog's estimate alone and
    the oracle."""
    import torch
    n, lmax = 48, 4
    cats = [small_catalogs(3000, 20000, L, seed=s) for s in (81, 82)]
    alone = [_alone(n, prec, lmax, d, r) for d, r in cats]
    refs = [_oracle(n, lmax, d, r) for d, r in cats]
    dev = [(_dev(d), _dev(r)) for d, r in cats]
    plans = [_plan(n, prec, lmax, stream=torch.cuda.Stream()) for _ in range(2)]
    for p in plans:
        p.prepare(lmax, _edges(n), 30000)
    busy = [None, None]
    got = []
    for i in range(6):
        j = i % 2
        if busy[j] is not None:
            got.append((busy[j], plans[j].finish()))
        plans[j].enqueue(*dev[i % 2])
        busy[j] = i % 2
    for j in range(2):
        got.append((busy[j], plans[j].finish()))
    assert len(got) == 6
    for c, res in got:
        _same(res, alone[c], prec, f"in flight cat={c} prec={prec}")
        assert _scaled_err(res, refs[c]) <= (1e-5 if prec == 0 else 1e-12)
    for p in plans:
        p.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_zero_normalisation_rejected(gpu, prec):
    """A catalog whose normalisation I vanishes (every random weight zero, or every data
    weight zero in a periodic box) has no estimate: painting, the asynchronous finish, a
    batch item and a served request report PKM_EINVAL, outputs untouched and the plan left
    unpainted; the next good paint on the same plan gives the estimate run alone."""
    import torch
    from paper_1704_02357_amd import Batch, PkmError, Server
    from synth import Catalog
    n, lmax = 32, 4
    d, r = small_catalogs(2000, 12000, L, seed=81)
    r0 = Catalog(r.pos, np.zeros(len(r.pos)), r.nbar)
    d0 = Catalog(d.pos, np.zeros(len(d.pos)), d.nbar)
    ref = _alone(n, prec, lmax, d, r)
    print(f"[case] zero normalisation prec={prec}: synchronous paint", flush=True)
    p = _plan(n, prec, lmax)
    for bad in ((d, r0), (d0, None)):
        with pytest.raises(PkmError) as e:
            p.paint(*bad)
        assert e.value.status == 1 and "normalisation" in str(e.value)
        with pytest.raises(PkmError) as e:
            p.compute_multipoles(lmax, _edges(n))
        assert e.value.status == 2
    p.paint(d, r)
    _same(p.compute_multipoles(lmax, _edges(n)), ref, prec, f"after rejected paint prec={prec}")
    p.close()

    print(f"[case] zero normalisation prec={prec}: enqueue / finish", flush=True)
    p = _plan(n, prec, lmax, stream=torch.cuda.Stream())
    p.prepare(lmax, _edges(n), 14000)
    dd, rr, rr0 = _dev(d), _dev(r), _dev(r0)
    p.enqueue(dd, rr0)
    with pytest.raises(PkmError) as e:
        p.finish()
    assert e.value.status == 1
    with pytest.raises(PkmError) as e:
        p.compute_multipoles(lmax, _edges(n))
    assert e.value.status == 2
    p.enqueue(dd, rr)
    _same(p.finish(), ref, prec, f"enqueue after rejected finish prec={prec}")

    print(f"[case] zero normalisation prec={prec}: batch", flush=True)
    q = _plan(n, prec, lmax, stream=torch.cuda.Stream())
    q.prepare(lmax, _edges(n), 14000)
    b = Batch()
    b.add(p, dd, rr0)
    b.add(q, dd, rr)
    b.run(use_graph=False)
    with pytest.raises(PkmError) as e:
        b.result(0)
    assert e.value.status == 1
    _same(b.result(1), ref, prec, f"batch item beside a rejected one prec={prec}")
    b.close()
    p.close()
    q.close()

    print(f"[case] zero normalisation prec={prec}: server", flush=True)
    sv = Server(max_inflight=2)
    kw = dict(observer=OBS, window=3, interlaced=True, compensated=True, precision=prec, ell_max_hint=lmax)
    bad = sv.submit(n, L, lmax, _edges(n), d, r0, **kw)
    good = sv.submit(n, L, lmax, _edges(n), d, r, **kw)
    with pytest.raises(PkmError) as e:
        sv.wait(bad)
    assert e.value.status == 1
    _same(sv.wait(good), ref, prec, f"served request beside a rejected one prec={prec}")
    sv.close()


def test_batch_uneven_mocks_graph_replays(gpu):
    """Six mocks on three mesh sizes (two plans per size, each on its own stream), issued
    directly and as one captured graph; replays with eager work in between, and a replay
    after a catalog's contents changed, all match the estimates run alone."""
    import torch
    from paper_1704_02357_amd import Batch
    prec, lmax = 0, 4
    sizes = [32, 48, 64, 32, 48, 64]
    mocks = [small_catalogs(1500 + 300 * i, 9000 + 1000 * i, L, seed=100 + i) for i in range(6)]
    plans = {}
    for n in sorted(set(sizes)):
        for k in range(2):
            p = _plan(n, prec, lmax, stream=torch.cuda.Stream())
            p.prepare(lmax, _edges(n), 20000)
            plans[(n, k)] = p
    b = Batch()
    dev = []
    for i, n in enumerate(sizes):
        d, r = mocks[i]
        dd, rr = _dev(d), _dev(r)
        dev.append((dd, rr))
        b.add(plans[(n, i % 2)], dd, rr)
    from tests.parity_util import assert_pole_parity
    refs = [_alone(n, prec, lmax, *mocks[i]) for i, n in enumerate(sizes)]
    orcs = [_oracle(n, lmax, *mocks[i]) for i, n in enumerate(sizes)]
    ms = b.run(use_graph=False)
    print(f"[batch] direct {ms:.2f} ms", flush=True)
    for i in range(6):
        _same(b.result(i), refs[i], prec, f"direct item {i}")
        assert_pole_parity(b.result(i), orcs[i], prec, f"direct item {i} vs oracle")
    for rep in range(3):
        ms = b.run(use_graph=True)
        print(f"[batch] graph replay {rep} {ms:.2f} ms", flush=True)
        for i in range(6):
            _same(b.result(i), refs[i], prec, f"graph replay {rep} item {i}")
            assert_pole_parity(b.result(i), orcs[i], prec, f"graph replay {rep} item {i} vs oracle")
        # eager work and synchronisation between replays
        x = torch.randn(1 << 20, device="cuda")
        torch.cuda.synchronize()
        assert torch.isfinite(x.sum()).item()
        _alone(32, prec, 2, *mocks[0])
    # new catalog contents at the same addresses and sizes: the graph reads them
    from synth import Catalog
    d2, r2 = small_catalogs(1500, 9000, L, seed=999)
    dd, rr = dev[0]
    dd[0].copy_(torch.tensor(d2.pos, device="cuda"))
    rr[0].copy_(torch.tensor(r2.pos, device="cuda"))
    torch.cuda.synchronize()
    b.run(use_graph=True)
    new_d = Catalog(d2.pos, mocks[0][0].w, mocks[0][0].nbar)
    new_r = Catalog(r2.pos, mocks[0][1].w, mocks[0][1].nbar)
    _same(b.result(0), _alone(32, prec, lmax, new_d, new_r), prec, "replay after new contents")
    b.close()
    for p in plans.values():
        p.close()


def test_server_mixed_stream_matches_alone(gpu):
    """Requests of different sizes, l_max, precision and with or without randoms, submitted
    at once: admitted while others run, overlapping on the device, each equal to its
    estimate run alone."""
    from paper_1704_02357_amd import Server
    reqs = []
    for i, (n, lmax, prec, with_r) in enumerate([(32, 4, 0, True), (48, 8, 0, True), (64, 2, 1, True),
                                                 (32, 4, 1, False), (64, 4, 0, True), (48, 4, 0, True),
                                                 (32, 6, 0, True), (64, 4, 0, True)]):
        d, r = small_catalogs(2000 + 500 * i, 12000 if with_r else 0, L, seed=300 + i)
        reqs.append((n, lmax, prec, d, r))
    sv = Server(max_inflight=3)
    tickets = [sv.submit(n, L, lmax, _edges(n), d, r, observer=OBS, window=3, interlaced=True, compensated=True,
                         precision=prec, ell_max_hint=lmax) for n, lmax, prec, d, r in reqs]
    got = [sv.wait(t) for t in tickets]
    st = sv.stats()
    print(f"[server] {st}", flush=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["max_concurrent"] >= 2
    assert st["resident_plans"] >= 3
    from tests.parity_util import assert_pole_parity
    for (n, lmax, prec, d, r), g in zip(reqs, got):
        _same(g, _alone(n, prec, lmax, d, r), prec, f"server n={n} l={lmax} prec={prec} randoms={r is not None}")
        assert_pole_parity(g, _oracle(n, lmax, d, r), prec, f"server n={n} l={lmax} prec={prec} vs oracle")
    sv.close()


def test_server_budget_admission(gpu):
    """Under a budget that holds one 64^3 plan, requests still complete (one at a time),
    the resident bytes never exceed the budget, and a request that cannot fit fails."""
    from paper_1704_02357_amd import PkmError, Server
    d, r = small_catalogs(2000, 12000, L, seed=5)
    probe = _plan(64, 0, 4, torch_allocator=False)
    probe.prepare(4, _edges(64), 14000)
    one = probe.stats()["device_bytes"]
    probe.close()
    budget = int(one * 1.6)
    sv = Server(max_inflight=4, hbm_budget_bytes=budget)
    ts = [sv.submit(64, L, 4, _edges(64), d, r, observer=OBS, precision=0, ell_max_hint=4,
                    box_origin=(-150.0 + 0.1 * k, -150.0, -150.0)) for k in range(3)]
    outs = [sv.wait(t) for t in ts]
    st = sv.stats()
    print(f"[server budget] budget={budget} {st}", flush=True)
    assert st["completed"] == 3 and st["peak_bytes"] <= budget
    assert all(np.isfinite(o["poles"][0]).any() for o in outs)
    big = sv.submit(128, L, 16, _edges(128), d, r, observer=OBS, precision=1, ell_max_hint=16)
    with pytest.raises(PkmError):
        sv.wait(big)
    sv.close()


SHAPES = {  # per mesh size: power-of-two and 3-smooth schedules
    64: [dict(e_col=4, tile=4, e_z=4, zlines=4, e_post=4, tile_post=2, paint_tile=4, post_axis=2),
         dict(e_col=8, tile=8, e_z=8, zlines=2, e_post=8, tile_post=4, paint_tile=16),
         dict(e_col=16, tile=2, e_post=4, tile_post=8, post_axis=2)],
    48: [dict(e_col=12, tile=4, e_z=6, zlines=8, e_post=6, tile_post=4, paint_tile=8, post_axis=2),
         dict(e_col=6, tile=8, e_z=12, zlines=2, e_post=12, tile_post=2, paint_tile=4),
         dict(e_col=6, tile=2, e_z=6, zlines=16, e_post=6, tile_post=8, post_axis=2)],
}


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [48, 64])
@pytest.mark.parametrize("si", range(3))
def test_shaped_plan_matches_oracle(gpu, prec, n, si):
    """Non-default launch shapes (generic kernels, other tiles, radix-3 schedules, the other
    post-pass axis) give the oracle's multipoles to the precision form's tolerance."""
    from oracle.estimator import multipoles
    from tests.parity_util import assert_pole_parity, oracle_params
    shape = dict(SHAPES[n][si])
    d, r = small_catalogs(3000, 20000, L, seed=400 + si)
    p = _plan(n, prec, 4, shape=shape)
    print(f"[shape] n={n} prec={prec} {p.shape()}", flush=True)
    assert p.shape()["post_axis"] == 2
    p.paint(d, r)
    got = p.compute_multipoles(4, _edges(n))
    ref = multipoles(d, r, oracle_params(n, L, OBS, 3, True, True), 4, _edges(n))
    assert_pole_parity(got, ref, prec, f"shape {si} n={n}")
    p.close()


def test_retired_post_axis_rejected(gpu):
    """The post-pass runs along y over kz-major field buffers: post_axis 1 (x) is refused."""
    from paper_1704_02357_amd import PkmError
    with pytest.raises(PkmError):
        _plan(64, 0, 4, shape=dict(post_axis=1))


def test_autotune_picks_valid_shape_and_caches(gpu, tmp_path):
    from paper_1704_02357_amd import autotune
    cache = str(tmp_path / "tune.json")
    kw = dict(observer=OBS, window=3, interlaced=True, compensated=True, precision=0)
    t = autotune(64, L, ell_max=4, n_particles=60000, reps=1, cache=cache, **kw)
    print(f"[autotune] {t}", flush=True)
    assert t["ms"] > 0 and t["default_ms"] > 0 and t["ms"] <= t["default_ms"] * 1.0000001
    shape = {k: v for k, v in t.items() if k not in ("ms", "default_ms")}
    p = _plan(64, 0, 4, shape=shape)
    assert p.shape() == shape
    d, r = small_catalogs(3000, 20000, L, seed=77)
    p.paint(d, r)
    _same(p.compute_multipoles(4, _edges(64)), _alone(64, 0, 4, d, r), 0, "tuned shape")
    p.close()
    assert autotune(64, L, ell_max=4, n_particles=60000, reps=1, cache=cache, **kw) == t


def test_batch_refuses_changed_plan(gpu):
    """A plan re-prepared after pkm_batch_add (larger ell_max: larger result slot, new
    tables and field buffers) makes the next run return PKM_EORDER before anything is
    issued, with or without a captured graph; items added again run and match alone."""
    import torch
    from paper_1704_02357_amd import Batch, PkmError
    n, prec = 32, 0
    d, r = small_catalogs(1500, 9000, L, seed=55)
    dd, rr = _dev(d), _dev(r)
    ref = _alone(n, prec, 4, d, r)
    for use_graph in (False, True):
        p = _plan(n, prec, 4, stream=torch.cuda.Stream())
        p.prepare(4, _edges(n), 20000)
        b = Batch()
        b.add(p, dd, rr)
        b.run(use_graph=use_graph)
        _same(b.result(0), ref, prec, f"before re-prepare graph={use_graph}")
        p.prepare(8, _edges(n), 20000)
        print(f"[case] batch after re-prepare graph={use_graph}", flush=True)
        with pytest.raises(PkmError) as e:
            b.run(use_graph=use_graph)
        assert e.value.status == 2 and "changed" in str(e.value)
        with pytest.raises(PkmError) as e:   # nothing ran: no result to read
            b.result(0)
        assert e.value.status == 2
        b.close()
        p.prepare(4, _edges(n), 20000)
        b = Batch()
        b.add(p, dd, rr)
        b.run(use_graph=use_graph)
        _same(b.result(0), ref, prec, f"items added again graph={use_graph}")
        b.close()
        p.close()


def test_particle_limit_rejected_before_device_work(gpu):
    """Catalog counts above PKM_MAX_PARTICLES are refused by paint, prepare and submit with
    PKM_EINVAL, before any array is read (the pointers here are never dereferenced)."""
    import ctypes as C
    from paper_1704_02357_amd import PkmError, Server
    from paper_1704_02357_amd.pkm import Catalog, MAX_PARTICLES
    p = _plan(32, 0, 4)
    fake = C.c_void_p(0x1000)
    big = Catalog(fake, None, fake, MAX_PARTICLES, 1)
    small = Catalog(fake, None, fake, 10, 1)
    assert p.lib.pkm_paint(p.h, C.byref(small), C.byref(big)) == 1
    assert "PKM_MAX_PARTICLES" in p.lib.pkm_plan_last_error(p.h).decode()
    with pytest.raises(PkmError) as e:
        p.prepare(4, _edges(32), MAX_PARTICLES + 1)
    assert e.value.status == 1
    p.close()
