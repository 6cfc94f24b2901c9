#!/usr/bin/env python3
"""Benchmark: P_l(k) estimates per second at 512^3, l <= 4, on one MI355X.

One step (= one estimate) is pkm_paint + pkm_compute_multipoles(ell_max=4) on a catalog
already resident in HBM: 1e6 lognormal galaxies + 2e7 randoms in a 2500 Mpc/h box, TSC with
interlacing and compensation, 64 uniform k bins up to the Nyquist frequency (17 transforms).
Prints one JSON line (rank 0).  The FP32 form gives `value`; the FP64 form is reported
beside it.  `roofline` covers the kernel stage with the largest device time, measured with
HIP events on the plan's stream inside the timed region.  `cpu_baseline` times the FP64
oracle on a bounded sample of the same estimate and scales it to estimates/s.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

METRIC = "P_ℓ(k) estimates/s at 512³ ℓ≤4 (FP32 vs FP64), HBM GB/s; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
NMESH, BOX, ELL_MAX = 512, 2500.0, 4
OBSERVER = (0.0, 0.0, -1500.0)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stage_bytes(nmesh: int, es: int, n_part: int, nfields: int) -> dict:
    """Algorithmic HBM bytes per estimate of each kernel stage: one read and one write of
    every element a pass must touch (X bytes per mesh or half spectrum, 40 bytes per
    catalog object read by the sums and the painter)."""
    X = es * nmesh ** 3          # half spectrum (N x N x N/2 complex) == real mesh bytes
    return {
        "sums": 40.0 * n_part,
        "fill": 2.0 * X,
        "paint": 40.0 * n_part + 2.0 * X,
        "zfwd": 4.0 * X,
        "ycol": 4.0 * X + 2.0 * nfields * X,
        "xcombine": 4.0 * X,
        "iycol": 2.0 * X,
        "zpre": (1.0 + nfields) * X,
        "xpost": (1.0 + nfields) * X,
        "reduce": 0.0,
    }


HERE = os.path.dirname(os.path.abspath(__file__))
# Sources whose change invalidates stored HBM counter readings of the transform kernels.
TRAFFIC_SOURCES = ["paper_1704_02357_amd/csrc/kernels_fft.hip", "paper_1704_02357_amd/csrc/device_common.hpp",
                   "paper_1704_02357_amd/csrc/kernels.hpp", "paper_1704_02357_amd/csrc/plan.hip"]


def source_digest() -> str:
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(stage: str):
    """HBM bytes per launch of a stage from a committed counter summary (profiles/*_traffic.txt,
    a line 'TRAFFIC {json}'), or None when there is none for the current kernel sources."""
    digest = source_digest()
    for path in sorted(glob.glob(os.path.join(HERE, "profiles", "*_traffic.txt"))):
        with open(path) as f:
            for line in f:
                if not line.startswith("TRAFFIC "):
                    continue
                rec = json.loads(line[len("TRAFFIC "):])
                if rec.get("stage") == stage and rec.get("source_digest") == digest and rec.get("nmesh") == NMESH:
                    return rec["hbm_bytes_per_launch"]
    return None


def summarize_profile(directory: str) -> None:
    """Print the per-kernel summary of a rocprofv3 CSV output directory: kernel statistics
    (--kernel-trace --stats) and/or counter means per dispatch (--pmc)."""
    def rows(pattern):
        out = []
        for path in sorted(glob.glob(os.path.join(directory, "**", pattern), recursive=True)):
            with open(path, newline="") as f:
                out.extend(csv.DictReader(f))
        return out

    def short(name):
        name = name.replace("(anonymous namespace)::", "").replace("pkm::", "")
        return name.split("(")[0].replace("void ", "")[:60]

    stats = rows("*kernel_stats.csv")
    if stats:
        print(f"{'kernel':60s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}")
        for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
            print(f"{short(r['Name']):60s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.1f} "
                  f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}")
    pmc = rows("*counter_collection.csv")
    if pmc:
        acc = {}
        for r in pmc:
            key = (short(r["Kernel_Name"]), r["Counter_Name"])
            a = acc.setdefault(key, [0.0, set()])
            a[0] += float(r["Counter_Value"])
            a[1].add(r["Dispatch_Id"])
        print(f"{'kernel':60s} {'counter':>14s} {'dispatches':>10s} {'mean_per_dispatch':>18s}")
        for (k, c), (v, d) in sorted(acc.items()):
            print(f"{k:60s} {c:>14s} {len(d):10d} {v / len(d):18.6g}")


def run_in_flight(plans, steps: int, data, rand):
    """Estimate i on plans[i mod len(plans)]: a plan's previous estimate is finished before its
    next one is enqueued, so up to len(plans) estimates are in flight, and every estimate
    enqueued is finished before returning.  Returns the last result and the number finished."""
    k = len(plans)
    busy = [False] * k
    res, done = None, 0
    for i in range(steps):
        j = i % k
        if busy[j]:
            res = plans[j].finish()
            done += 1
        plans[j].enqueue(data, rand)
        busy[j] = True
    for i in range(steps, steps + k):  # drain in enqueue order
        j = i % k
        if busy[j]:
            res = plans[j].finish()
            done += 1
            busy[j] = False
    return res, done


def run_form(precision: int, data, rand, edges, steps: int, warmup: int, pipeline: int = 2):
    """Estimates through the asynchronous calls: pkm_prepare once per plan, then per step
    pkm_enqueue (paint, every transform, all (l, m) fields, binning; no host wait inside) and
    pkm_finish (wait, normalise).  The headline loop keeps `pipeline` estimates in flight, each
    on its own plan and stream (step i on plan i mod pipeline, whose previous estimate is
    finished first), so the latency-bound painting of one estimate overlaps the transforms of
    another; per-launch timing is off.  A serial loop on one plan gives the per-estimate latency
    and the one-in-flight rate; a third loop of the same steps on that plan records HIP events
    around every launch and gives the per-stage device times (and its own wall time, to show the
    events' overhead)."""
    import torch
    from paper_1704_02357_amd import Plan
    pipeline = max(1, pipeline)
    plans = [Plan(NMESH, BOX, observer=OBSERVER, window=3, interlaced=True, compensated=True, precision=precision,
                  ell_max_hint=ELL_MAX, stream=torch.cuda.Stream()) for _ in range(pipeline)]
    for p in plans:
        p.prepare(ELL_MAX, edges, int(data[0].shape[0] + rand[0].shape[0]))
        p.set_stage_timing(False)
    for _ in range(warmup):
        for p in plans:
            p.enqueue(data, rand)
        for p in plans:
            res = p.finish()
    plan = plans[0]
    # one estimate in flight: latency and rate
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        plan.enqueue(data, rand)
        res = plan.finish()
        lat.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    sec_one = time.perf_counter() - t0
    # headline: `pipeline` estimates in flight
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, done = run_in_flight(plans, steps, data, rand)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert done == steps
    # stage pass: the same steps on one plan with per-launch events
    plan.reset_stats()
    plan.set_stage_timing(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        plan.enqueue(data, rand)
        plan.finish()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    st = plan.stats()
    for p in plans:
        p.close()
    return res, (t1 - t0), np.array(lat), st, (t3 - t2), sec_one


def golden_poles(info, data, rand):
    """The FP64 oracle's P_l(k) for this workload from tests/golden/workload_512_l4_poles.txt
    (written by tests/golden/make_workload_golden.py from the oracle only), after checking that
    the catalog digest and sizes match the inputs of this run; None otherwise."""
    from synth import catalog_digest
    path = os.path.join(HERE, "tests", "golden", "workload_512_l4_poles.txt")
    if not os.path.exists(path):
        return None
    head, rows = {}, []
    with open(path) as f:
        for line in f:
            if line.startswith("# catalog:"):
                toks = line.split()
                head["n_data"] = int(toks[toks.index("n_data") + 1].rstrip(","))
                head["n_rand"] = int(toks[toks.index("n_rand") + 1].rstrip(","))
                head["digest"] = toks[toks.index("digest") + 1]
            elif line.startswith("# shot_noise"):
                head["shot_noise"] = float(line.split()[-1])
            elif not line.startswith("#") and line.strip():
                rows.append([float(v) for v in line.split()])
    if head.get("n_data") != info["n_data"] or head.get("n_rand") != info["n_rand"]:
        return None
    if head.get("digest") != catalog_digest(data, rand):
        return None
    a = np.array(rows)
    return {"poles": a[:, 4:7].T.copy(), "n_modes": a[:, 2].astype(np.int64), "shot_noise": head["shot_noise"],
            "edges": np.concatenate([a[:, 0], a[-1:, 1]])}


def err_vs_oracle(res, ref) -> dict:
    """Largest per-bin error of a result against the oracle: scaled by max(|P_l|, P_0 + S)
    (the parity tests' pass rule) and plain relative."""
    po, pg = ref["poles"], np.asarray(res["poles"])
    raw0 = po[0] + ref["shot_noise"]
    scale = np.maximum(np.abs(po), np.abs(raw0)[None, :])
    ok = np.isfinite(po)
    rel = np.abs(pg - po)[ok] / np.abs(po)[ok]
    return {"max_scaled": float(np.max(np.abs(pg - po)[ok] / scale[ok])), "max_plain_rel": float(np.max(rel)),
            "n_modes_equal": bool(np.array_equal(np.asarray(res["n_modes"]), ref["n_modes"]))}


def catalog_upload(data, rand, dst) -> dict:
    """Host-to-device copy of the catalog arrays (positions, weights, n-bar of both catalogs)
    into the resident device buffers: from pageable numpy memory and from pinned memory; the
    median of three copies each.  Not part of the estimate's timed region."""
    import torch
    host = [np.ascontiguousarray(a, dtype=np.float64) for a in (data.pos, data.w, data.nbar, rand.pos, rand.w, rand.nbar)]
    nbytes = sum(a.nbytes for a in host)
    pinned = [torch.from_numpy(a).pin_memory() for a in host]
    out = {"bytes": int(nbytes)}
    for name, srcs in (("pageable", [torch.from_numpy(a) for a in host]), ("pinned", pinned)):
        ms = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for d, h in zip(dst, srcs):
                d.copy_(h.view_as(d), non_blocking=(name == "pinned"))
            torch.cuda.synchronize()
            ms.append(1e3 * (time.perf_counter() - t0))
        out[f"ms_{name}"] = round(float(np.median(ms)), 3)
        out[f"GBps_{name}"] = round(nbytes / (np.median(ms) * 1e-3) / 1e9, 1)
    del pinned
    return out


def fft_bench(args) -> dict:
    """The library's 3D real-to-complex transform (the one pkm_paint applies to each painted
    mesh) against ROCm's FFT library through torch.fft.rfftn, same sizes and precisions, device
    time per transform; for comparison only (the estimator never calls the library FFT)."""
    import torch
    from paper_1704_02357_amd import Plan
    rows = []
    for n in (256, 512, 1024):
        for prec in (0, 1):
            rdt, cdt = (torch.float64, torch.complex128) if prec else (torch.float32, torch.complex64)
            g = torch.Generator(device="cuda")
            g.manual_seed(n + prec)
            x = torch.randn((n, n, n), generator=g, dtype=rdt, device="cuda")
            plan = Plan(n, 1000.0, precision=prec)
            ours = torch.empty((n, n, n // 2), dtype=cdt, device="cuda")

            def timed(fn, reps):
                fn()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    fn()
                e1.record()
                torch.cuda.synchronize()
                return e0.elapsed_time(e1) / reps

            reps = 20 if n <= 512 else 5
            ms_ours = timed(lambda: plan.fft3d_forward(x, ours), reps)
            ref = {}
            ms_lib = timed(lambda: ref.__setitem__("y", torch.fft.rfftn(x)), reps)
            y = ref["y"][:, :, : n // 2]
            err = float((ours - y).abs().max() / y.abs().max())
            # algorithmic bytes of one R2C transform: the real input read, the half spectrum written
            byts = x.numel() * x.element_size() + ours.numel() * ours.element_size()
            rows.append({"n": n, "precision": "f64" if prec else "f32", "ms_ours": round(ms_ours, 3),
                         "ms_library": round(ms_lib, 3), "ours_over_library": round(ms_lib / ms_ours, 3),
                         "ours_GBps_in_plus_out": round(byts / (ms_ours * 1e-3) / 1e9, 1),
                         "max_rel_diff": err})
            log(f"[fft] {rows[-1]}")
            plan.close()
            del x, ours, ref, y
            torch.cuda.empty_cache()
    return {"metric": "3D R2C transform device time, this library against ROCm's FFT (torch.fft.rfftn)",
            "unit": "ms", "higher_is_better": False, "n_gpus": 1, "rows": rows,
            "data": "synthetic (standard normal real meshes)",
            "config": {"workload": "N^3 real to half spectrum, N = 256, 512, 1024, FP32 and FP64"}}


def cpu_baseline(data, rand, edges, workers: int) -> dict:
    """FP64 oracle timed on a bounded sample of one estimate, scaled to estimates/s.

    Sample: painting split into a per-cell part and a per-particle part, from two paints of
    catalog subsamples (1/10 and 1/40) onto a 256^3 mesh (per-cell part x8 for 512^3, the
    per-particle part extrapolated to the whole catalog); one full-grid forward transform (x17
    transforms); the harmonic weighting of one field on 1/4 of the nodes and of the modes
    (x4 x14 fields); one binning pass (x3 multipoles).  About 10-20 s of host work."""
    import scipy.fft as sfft
    from oracle.estimator import default_params, k_thresholds, mode_bins, node_vectors, mode_vectors, binned_sums
    from oracle.mesh import fkp_meshes
    from oracle.catalog import catalog_scalars
    from oracle.ylm import real_ylm
    from synth import Catalog
    p = default_params(NMESH, BOX, observer=OBSERVER, window=3, interlaced=True, compensated=True)
    slab_div = 4
    nfields = sum(2 * l + 1 for l in range(2, ELL_MAX + 1, 2))
    t = {}

    def paint_time(frac, nm):
        sub_d = Catalog(data.pos[::frac], data.w[::frac], data.nbar[::frac])
        sub_r = Catalog(rand.pos[::frac], rand.w[::frac], rand.nbar[::frac])
        t0 = time.perf_counter()
        sc = catalog_scalars(sub_d, sub_r, BOX)
        meshes = fkp_meshes(sub_d, sub_r, sc["alpha"], nm, BOX, p["box_origin"], 3, True)
        return time.perf_counter() - t0, meshes[0]

    ta, m = paint_time(10, NMESH // 2)
    tb, _ = paint_time(40, NMESH // 2)
    per_catalog = max(0.0, (ta - tb) / (1 / 10 - 1 / 40))
    per_mesh = max(0.0, ta - per_catalog / 10) * 8
    t["paint"] = per_mesh + per_catalog
    # a 512^3 density for the transform and field samples (the 256^3 mesh, each cell split in 8)
    d1 = m.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)
    del m
    t0 = time.perf_counter()
    c = sfft.fftn(d1, workers=workers)
    t["fft"] = (time.perf_counter() - t0) * (nfields + 3)
    xv = node_vectors(NMESH, BOX, p["box_origin"], p["observer"])
    kv = mode_vectors(NMESH)
    sl = NMESH // slab_div
    t0 = time.perf_counter()
    weighted = d1[:sl] * real_ylm(2, 1, xv[:sl])
    a = real_ylm(2, 1, kv[:sl]) * c[:sl]
    t["field"] = (time.perf_counter() - t0) * slab_div * nfields
    del xv, kv, weighted
    t0 = time.perf_counter()
    bins = mode_bins(NMESH, k_thresholds(edges, BOX))
    q = np.real(c * np.conj(c))
    binned_sums(q, bins, len(edges) - 1)
    t["bin"] = (time.perf_counter() - t0) * 3
    sec = sum(t.values())
    return {"value": 1.0 / sec, "unit": "estimates/s", "cores": workers, "kind": "oracle",
            "sample": f"FP64 numpy/scipy oracle: paint cost from 1/10 and 1/40 catalog subsamples on a 256^3 mesh "
                      f"(per-cell part x8, per-particle part extrapolated to the catalog), one 512^3 complex "
                      f"FFT (x{nfields + 3}), Y_lm(x) and Y_lm(k) weighting of one field on 1/{slab_div} of the "
                      f"grid (x{slab_div} x{nfields}), one binning pass (x3); seconds per estimate {sec:.1f} = "
                      + ", ".join(f"{k} {v:.1f}" for k, v in t.items())}


def batch_bench(args) -> dict:
    """64 seeded lognormal covariance mocks of uneven size (Nmesh 128/256/384 in turn,
    5e4-8e5 galaxies, 10x randoms), l <= 4, FP32: all mocks issued as one batch over
    per-plan streams, replayed as one HIP graph; against the same mocks run one by one."""
    import torch
    from paper_1704_02357_amd import Batch, Plan
    from synth import batch_mock
    n_mocks, lmax, per_size = args.mocks, 4, args.plans_per_size
    t0 = time.perf_counter()
    mocks = [batch_mock(i) for i in range(n_mocks)]
    log(f"[batch] {n_mocks} mocks generated in {time.perf_counter() - t0:.1f} s")
    dev = lambda a: None if a is None else torch.tensor(a, dtype=torch.float64, device="cuda")
    L = 2000.0
    edges = {n: np.arange(int(math.floor(math.pi * n / L / 0.01)) + 1, dtype=np.float64) * 0.01
             for n in (128, 256, 384)}
    plans = {}
    maxp = {}
    for d, r, info, n in mocks:
        maxp[n] = max(maxp.get(n, 0), len(d.pos) + len(r.pos))
    for n in sorted(maxp):
        for k in range(per_size):
            p = Plan(n, L, observer=OBSERVER, window=3, interlaced=True, compensated=True, precision=0,
                     ell_max_hint=lmax, stream=torch.cuda.Stream())
            p.prepare(lmax, edges[n], maxp[n])
            plans[(n, k)] = p
    b = Batch()
    cats = []
    count = {}
    for i, (d, r, info, n) in enumerate(mocks):
        dd = (dev(d.pos), dev(d.w), dev(d.nbar))
        rr = (dev(r.pos), dev(r.w), dev(r.nbar))
        cats.append((dd, rr))
        k = count.get(n, 0)
        count[n] = k + 1
        b.add(plans[(n, k % per_size)], dd, rr)
    torch.cuda.synchronize()
    b.run(use_graph=False)
    t_direct = min(b.run(use_graph=False) for _ in range(2))
    b.run(use_graph=True)   # capture + first replay
    t_graph = [b.run(use_graph=True) for _ in range(args.steps)]
    # the same mocks one after another through the synchronous calls (one plan per size)
    seq = {n: Plan(n, L, observer=OBSERVER, window=3, interlaced=True, compensated=True, precision=0,
                   ell_max_hint=lmax) for n in maxp}
    errs = []
    model_bytes = 0.0
    by_size = {}  # n -> [estimates, device ms, model bytes]
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    for i, (d, r, info, n) in enumerate(mocks):
        seq[n].paint(cats[i][0], cats[i][1])
        ref = seq[n].compute_multipoles(lmax, edges[n])
        st = seq[n].stats()
        mb = st["model_bytes_paint"] + st["model_bytes_compute"]
        model_bytes += mb
        acc = by_size.setdefault(n, [0, 0.0, 0.0])
        acc[0] += 1
        acc[1] += st["ms_paint"] + st["ms_compute"]
        acc[2] += mb
        got = b.result(i)
        scale = np.maximum(np.abs(ref["poles"]), np.abs(ref["poles"][0] + ref["shot_noise"])[None, :])
        ok = np.isfinite(ref["poles"])
        errs.append(float(np.max(np.abs(got["poles"] - ref["poles"])[ok] / scale[ok])))
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - s0) * 1e3
    med = float(np.median(t_graph))
    sizes_out = {str(n): {"estimates": a[0], "ms_per_estimate_sync": round(a[1] / a[0], 3),
                          "model_gb_per_s_sync": round(a[2] / (a[1] * 1e-3) / 1e9, 1)}
                 for n, a in sorted(by_size.items())}
    for p in list(plans.values()) + list(seq.values()):
        p.close()
    b.close()
    return {"metric": "covariance-mock P_l(k) estimates/s (64 lognormal mocks, Nmesh 128/256/384, l<=4, FP32, "
                      "one graph launch)",
            "value": round(n_mocks / (med * 1e-3), 2), "unit": "estimates/s", "n_gpus": 1, "steps": args.steps,
            "ms_per_batch_graph": round(med, 2), "ms_per_batch_direct": round(t_direct, 2),
            "ms_per_batch_sequential_sync": round(t_seq, 2),
            "model_gb_per_batch": round(model_bytes / 1e9, 2),
            "model_gb_per_s_graph": round(model_bytes / (med * 1e-3) / 1e9, 1),
            "per_size": sizes_out, "higher_is_better": True, "dtype": "f32",
            "data": "synthetic (seeded lognormal mocks, resident in HBM)",
            "config": {"workload": f"{n_mocks} mocks, Nmesh cycling 128/256/384, L=2000 Mpc/h, 5e4-8e5 galaxies, "
                                   "10x randoms, TSC + interlacing + compensation, l<=4, 0.01 h/Mpc bins",
                       "plans_per_size": per_size,
                       "hip_hw_queues": os.environ.get("GPU_MAX_HW_QUEUES", "runtime default")},
            "max_scaled_err_vs_sequential": max(errs)}


def sizes_bench(args) -> dict:
    """The radix-3 mesh sizes of the batch and serving workloads, one estimate at a time in
    both forms: Nmesh 384 (L = 2000 Mpc/h, a covariance mock of 8e5 galaxies) and 768
    (L = 2500 Mpc/h, 3e6 galaxies, the largest served catalog), 10x randoms, TSC + interlacing
    + compensation, l <= 4.  Device time of paint and multipoles per estimate (the last of
    `steps` after `warmup`), the byte model's rate, and the per-stage times of one more
    estimate with per-launch timing on."""
    import torch
    from paper_1704_02357_amd import Plan
    from synth import SurveyGeometry, lognormal_survey
    rows = []
    for n, box, ngal in ((384, 2000.0, 800_000), (768, 2500.0, 3_000_000)):
        d, r, _ = lognormal_survey(SurveyGeometry(box_len=box), ngal, 2000 + n, ng=256)
        log(f"[sizes] {n}^3: {len(d.pos)} galaxies, {len(r.pos)} randoms")
        dev = lambda c: (torch.tensor(c.pos, device="cuda"), torch.tensor(c.w, device="cuda"),
                         torch.tensor(c.nbar, device="cuda"))
        dd, rr = dev(d), dev(r)
        edges = np.arange(int(math.floor(math.pi * n / box / 0.01)) + 1, dtype=np.float64) * 0.01
        for prec in (0, 1):
            p = Plan(n, box, observer=OBSERVER, window=3, interlaced=True, compensated=True, precision=prec,
                     ell_max_hint=4)
            for _ in range(args.warmup + args.steps):
                p.paint(dd, rr)
                p.compute_multipoles(4, edges)
            st = p.stats()
            p.set_stage_timing(True)
            p.reset_stats()
            p.paint(dd, rr)
            p.compute_multipoles(4, edges)
            stages = {k: round(v, 3) for k, v in p.stats()["stage_ms"].items() if v > 0}
            shape = p.shape()
            p.close()
            ms = st["ms_paint"] + st["ms_compute"]
            gb = (st["model_bytes_paint"] + st["model_bytes_compute"]) / 1e9
            rows.append({"nmesh": n, "dtype": "f64" if prec else "f32", "ms_paint": round(st["ms_paint"], 3),
                         "ms_multipoles": round(st["ms_compute"], 3), "model_gb": round(gb, 2),
                         "model_gb_per_s": round(gb / (ms * 1e-3), 1), "stage_ms": stages, "shape": shape})
            log(f"[sizes] {rows[-1]}")
    return {"metric": "P_l(k) estimates/s at the radix-3 sizes (384^3, 768^3, l<=4), per form",
            "value": round(1e3 / (rows[0]["ms_paint"] + rows[0]["ms_multipoles"]), 2), "unit": "estimates/s (384^3 FP32)",
            "higher_is_better": True, "n_gpus": 1, "dtype": "f32+f64", "data": "synthetic (seeded lognormal surveys)",
            "config": {"workload": "384^3 (L=2000, 8e5 galaxies) and 768^3 (L=2500, 3e6 galaxies), 10x randoms, "
                                   "TSC + interlacing + compensation, l<=4, dk=0.01"},
            "rows": rows}


def basis_bench(args) -> dict:
    """Sec. 2.1's transform-count comparison measured as device time: the multipole pass
    (everything after painting) of the 512^3 workload through the spherical-harmonic
    decomposition and through the Cartesian one, l <= 4 and l <= 16, on one painted plan."""
    import torch
    from paper_1704_02357_amd import CARTESIAN, SPHERICAL, Plan
    from synth import config_c2
    data, rand, info = config_c2(n_gal=args.ngal, random_factor=args.random_factor)
    n, L = 512, 2500.0
    edges = np.arange(int(math.floor(math.pi * n / L / 0.01)) + 1, dtype=np.float64) * 0.01
    rows = []
    for prec in (0, 1):
        # 64 weighted fields resident at a time, the same for both decompositions
        plan = Plan(n, L, observer=OBSERVER, window=3, interlaced=True, compensated=True, precision=prec,
                    ell_max_hint=16, max_group=64)
        plan.paint(data, rand)
        for lmax in (4, 16):
            for basis, name in ((SPHERICAL, "spherical"), (CARTESIAN, "cartesian")):
                reps = max(1, min(args.steps, 10 if lmax == 4 else 3))
                r = plan.compute_multipoles(lmax, edges, basis=basis)   # warm-up (tables, buffers)
                ms = []
                for _ in range(reps):
                    r = plan.compute_multipoles(lmax, edges, basis=basis)
                    ms.append(plan.stats()["ms_compute"])
                nf = r["n_transforms"] - 3
                rows.append({"precision": "f64" if prec else "f32", "ell_max": lmax, "basis": name,
                             "weighted_fields": nf, "ms_compute": round(float(np.median(ms)), 3),
                             "ms_per_field": round(float(np.median(ms)) / nf, 4)})
                log(f"[basis] {rows[-1]}")
        plan.close()
        torch.cuda.empty_cache()
    ratios = {}
    for prec in ("f32", "f64"):
        for lmax in (4, 16):
            sp = next(x for x in rows if x["precision"] == prec and x["ell_max"] == lmax and x["basis"] == "spherical")
            ca = next(x for x in rows if x["precision"] == prec and x["ell_max"] == lmax and x["basis"] == "cartesian")
            ratios[f"{prec}_l{lmax}"] = {"fields_ratio": round(ca["weighted_fields"] / sp["weighted_fields"], 3),
                                         "time_ratio": round(ca["ms_compute"] / sp["ms_compute"], 3)}
    return {"metric": "multipole-pass device time by decomposition of L_l (512^3, after painting)",
            "unit": "ms", "higher_is_better": False, "n_gpus": 1, "rows": rows, "cartesian_over_spherical": ratios,
            "data": "synthetic (seeded lognormal survey mock, resident in HBM)",
            "config": {"workload": "512^3 mesh, L=2500 Mpc/h, 1e6 galaxies + 2e7 randoms, TSC + interlacing + "
                                   "compensation, 0.01 h/Mpc bins, at most 64 weighted fields resident"}}


def covariance_study(n: int = 128, box_len: float = 1000.0, n_mocks: int = 1000, beta: float = 0.35,
                     k_range=(0.1, 0.35), n_plans: int = 4, per_plan: int = 8, seed0: int = 10_000,
                     theory=None) -> dict:
    """Sec. 4.1 on the GPU: Gaussian Kaiser mocks (synth.kaiser) estimated to l <= 16 in batches
    replayed as one HIP graph, wedges from l <= 4 and l <= 16 with uniform and non-uniform mu
    bins (9 each), their correlation matrices over the mocks (averaged over the k bins in
    k_range) against linear theory (eq. gamma), and condition numbers for N_mu = l_max/2 + 1.

    theory: None (the library's host functions) or a pair (gamma, wedges) with the signatures
    gamma(l_max, mu_edges, beta) and wedges(poles, l_max, mu_edges), used for the theory
    matrices and for turning the measured multipoles into wedges."""
    import torch
    from paper_1704_02357_amd import NGP, Batch, Plan, kaiser_wedge_gamma, nonuniform_mu_edges, wedges
    if theory is not None:
        kaiser_wedge_gamma, wedges = theory
    from synth.kaiser import KaiserBox, node_positions
    far = (0.0, 0.0, -1.0e9)   # line of sight along z everywhere
    edges = np.arange(int(math.floor(math.pi * n / box_len / 0.01)) + 1, dtype=np.float64) * 0.01
    kb = KaiserBox(n, box_len, beta, device="cuda")
    pos = node_positions(n, box_len, device="cuda")
    plans = []
    for _ in range(n_plans):
        p = Plan(n, box_len, observer=far, window=NGP, interlaced=False, compensated=False, precision=0,
                 ell_max_hint=16, stream=torch.cuda.Stream())
        p.prepare(16, edges, n ** 3)
        plans.append(p)
    nb = n_plans * per_plan
    wbuf = [torch.empty(n ** 3, dtype=torch.float64, device="cuda") for _ in range(nb)]
    b = Batch()
    for i in range(nb):
        b.add(plans[i % n_plans], (pos, wbuf[i], None))
    poles = []
    t_gpu, t_gen = 0.0, 0.0
    done = 0
    while done < n_mocks:
        m = min(nb, n_mocks - done)
        t0 = time.perf_counter()
        for i in range(nb):
            kb.weights(seed0 + done + min(i, m - 1), out=wbuf[i])
        torch.cuda.synchronize()
        t_gen += time.perf_counter() - t0
        t_gpu += b.run(use_graph=True)
        for i in range(m):
            poles.append(b.result(i)["poles"])
        done += m
    for p in plans:
        p.close()
    b.close()
    poles = np.stack(poles)                       # (mocks, 9, nk)
    kc = 0.5 * (edges[:-1] + edges[1:])
    sel = (kc >= k_range[0]) & (kc <= k_range[1])
    schemes = {"uniform": np.linspace(0.0, 1.0, 10), "nonuniform": nonuniform_mu_edges(16)}

    def corr(c):
        d = np.sqrt(np.diag(c))
        return c / d[:, None] / d[None, :]

    def mean_norm_cov(w):                          # w: (mocks, nk_sel, nmu)
        acc = 0.0
        for j in range(w.shape[1]):
            c = np.cov(w[:, j, :], rowvar=False)
            acc = acc + c / np.trace(c)
        return acc / w.shape[1]

    corr_out = {}
    for lmax in (4, 16):
        for name, mu in schemes.items():
            w = np.stack([wedges(pl[: lmax // 2 + 1], lmax, mu) for pl in poles])[:, sel, :]
            rho = np.mean([corr(np.cov(w[:, j, :], rowvar=False)) for j in range(w.shape[1])], axis=0)
            th = corr(kaiser_wedge_gamma(lmax, mu, beta))
            off = ~np.eye(th.shape[0], dtype=bool)
            corr_out[f"l{lmax}_{name}"] = {"max_abs_diff_vs_linear_theory": round(float(np.max(np.abs(rho - th))), 4),
                                           "mean_abs_offdiag_measured": round(float(np.mean(np.abs(rho[off]))), 4),
                                           "mean_abs_offdiag_theory": round(float(np.mean(np.abs(th[off]))), 4)}
    cond = {}
    for lmax in range(4, 17, 2):
        for name, mu in (("uniform", np.linspace(0.0, 1.0, lmax // 2 + 2)), ("nonuniform", nonuniform_mu_edges(lmax))):
            w = np.stack([wedges(pl[: lmax // 2 + 1], lmax, mu) for pl in poles])[:, sel, :]
            g = kaiser_wedge_gamma(lmax, mu, beta)
            sv_t = np.linalg.svd(g, compute_uv=False)
            sv_m = np.linalg.svd(mean_norm_cov(w), compute_uv=False)
            cond[f"l{lmax}_{name}"] = {"theory": float("%.4g" % (sv_t[0] / sv_t[-1])),
                                       "measured": float("%.4g" % (sv_m[0] / sv_m[-1]))}
    return {"mocks": int(n_mocks), "nmesh": n, "box_len": box_len, "beta": beta, "k_range": list(k_range),
            "k_bins_used": int(sel.sum()), "ms_gpu_total": round(t_gpu, 1), "s_generate_total": round(t_gen, 2),
            "estimates_per_s_gpu": round(n_mocks / (t_gpu * 1e-3), 1), "correlation": corr_out,
            "condition_number": cond}


def covariance_bench(args) -> dict:
    out = covariance_study(n_mocks=args.cov_mocks)
    return {"metric": "Kaiser-mock wedge covariance: l<=16 estimates/s through one graph per batch (128^3)",
            "value": out["estimates_per_s_gpu"], "unit": "estimates/s", "higher_is_better": True, "n_gpus": 1,
            "dtype": "f32", "data": "synthetic (Gaussian linear-Kaiser fields on the mesh nodes, generated on the GPU)",
            "config": {"workload": f"{out['mocks']} mocks, 128^3 mesh, L=1000 Mpc/h, beta=0.35, NGP, line of sight z, "
                                   "l<=16, 9 uniform / 9 non-uniform wedges"}, **out}


def serve_pool(n_catalogs: int, random_factor: float):
    """The serving workload's catalog pool: seeded lognormal surveys (L = 2500 Mpc/h, seeds
    3000 + j) with N_gal log-uniform in [1e5, 3e6] and random_factor x randoms, generated on
    host threads."""
    from concurrent.futures import ThreadPoolExecutor
    from synth import SurveyGeometry, lognormal_survey
    geom = SurveyGeometry(box_len=2500.0)
    ngal = np.exp(np.random.default_rng(3000).uniform(math.log(1e5), math.log(3e6), n_catalogs))
    done = [0]

    def one(j):
        d, r, _ = lognormal_survey(geom, int(ngal[j]), 3000 + j, ng=128, random_factor=random_factor, workers=2)
        done[0] += 1
        log(f"[serve] catalog {j}: {len(d.pos)} galaxies, {len(r.pos)} randoms ({done[0]} of {n_catalogs} done)")
        return d, r

    with ThreadPoolExecutor(max_workers=8) as ex:
        return list(ex.map(one, range(n_catalogs)))


def serve_bench(args) -> dict:
    """Serving workload in one precision form: a pool of registered catalogs, requests that
    each pick a catalog, Nmesh in {256, 384, 512, 768} and l_max in {4, 8, 16} uniformly.
    The capacity is measured first by a closed burst (every request queued at once); then
    Poisson streams arrive at the given fractions of that capacity, each reporting
    throughput and p50/p99 latency (submit to result)."""
    from paper_1704_02357_amd import Server
    prec = args.serve_precision
    L = 2500.0
    t0 = time.perf_counter()
    pool = serve_pool(args.catalogs, args.serve_random_factor)
    log(f"[serve] pool of {len(pool)} catalogs generated in {time.perf_counter() - t0:.0f} s")
    sizes, lmaxes = [256, 384, 512, 768], [4, 8, 16]
    sv = Server(max_inflight=args.inflight, field_group=args.field_group)
    ids = [sv.register_catalog(d, r) for d, r in pool]
    n_obj = sum(len(d.pos) + len(r.pos) for d, r in pool)
    reg = sv.stats()["registered_bytes"]
    log(f"[serve] {len(ids)} catalogs registered, {n_obj} objects, {reg / 2 ** 30:.1f} GiB resident")
    del pool
    rng = np.random.default_rng(2026 + prec)

    def draw(k):
        out = []
        for _ in range(k):
            n, lmax = int(rng.choice(sizes)), int(rng.choice(lmaxes))
            edges = np.arange(int(math.floor(math.pi * n / L / 0.01)) + 1, dtype=np.float64) * 0.01
            out.append((n, lmax, int(rng.integers(0, len(ids))), edges))
        return out

    def submit(req):
        n, lmax, j, edges = req
        return sv.submit(n, L, lmax, edges, catalog_id=ids[j], observer=OBSERVER, window=3, interlaced=True,
                         compensated=True, precision=prec, ell_max_hint=lmax)

    def stream(reqs, rate, label):
        """Submit at Poisson arrivals (rate 0: all at once) from a thread; wait for all.  The
        server's statistics are reset first, so latency covers this stream only."""
        import threading
        sv.reset_stats()
        gaps = rng.exponential(1.0 / rate, size=len(reqs)) if rate > 0 else np.zeros(len(reqs))
        tickets = [None] * len(reqs)

        def submitter():
            start, due = time.perf_counter(), 0.0
            for i, rq in enumerate(reqs):
                due += gaps[i]
                delay = start + due - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                tickets[i] = (submit(rq), time.perf_counter())

        s0 = time.perf_counter()
        th = threading.Thread(target=submitter)
        th.start()
        done = 0
        while done < len(reqs):
            while tickets[done] is None:
                time.sleep(0.001)
            sv.wait(tickets[done][0])
            done += 1
            if done % 50 == 0:
                log(f"[serve] {label}: {done} of {len(reqs)} results at {time.perf_counter() - s0:.0f} s")
        th.join()
        wall = time.perf_counter() - s0
        st = sv.stats()
        form = "fp64" if prec else "fp32"
        return {"requests": len(reqs), "arrival_rate_per_s": round(rate, 3), "wall_s": round(wall, 2),
                "served_per_s": round(len(reqs) / wall, 3), "completed": st["completed"], "failed": st["failed"],
                "latency_ms": {"p50": round(st[f"latency_p50_ms_{form}"], 2),
                               "p99": round(st[f"latency_p99_ms_{form}"], 2), "mean": round(st["latency_mean_ms"], 2)},
                "max_concurrent": st["max_concurrent"], "mesh_reuses": st["mesh_reuses"]}

    # warm the plan pool (one request per (N, l_max) configuration), then the capacity burst
    warm = [(n, lmax, k % len(ids), np.arange(int(math.floor(math.pi * n / L / 0.01)) + 1, dtype=np.float64) * 0.01)
            for k, (n, lmax) in enumerate((n, l) for n in sizes for l in lmaxes)]
    for rq in warm:
        sv.wait(submit(rq))
    log(f"[serve] plan pool warmed: {sv.stats()['resident_plans']} plans")
    burst = stream(draw(args.burst), 0.0, "capacity burst")
    capacity = burst["served_per_s"]
    log(f"[serve] capacity {capacity:.3f} requests/s")
    runs = []
    for frac in args.load_fractions:
        n_req = args.requests if abs(frac - 0.8) < 1e-9 else args.sweep_requests
        if args.stream_seconds:  # shorten the stream to about that many seconds of arrivals
            n_req = max(20, min(n_req, int(args.stream_seconds * frac * capacity)))
        runs.append(dict(stream(draw(n_req), frac * capacity, f"stream at {frac} x capacity"), load_fraction=frac))
        log(f"[serve] {runs[-1]}")
    st = sv.stats()
    sv.close()
    main = next((r for r in runs if abs(r["load_fraction"] - 0.8) < 1e-9), runs[0] if runs else burst)
    form = "fp64" if prec else "fp32"
    return {"metric": f"served P_l(k) requests/s, {form.upper()} form (Poisson stream at 0.8 x capacity), "
                      "p50/p99 latency",
            "value": main["served_per_s"], "unit": "requests/s", "n_gpus": 1, "higher_is_better": True,
            "latency_ms": main["latency_ms"], "capacity_per_s": capacity, "capacity_burst": burst, "streams": runs,
            "server": {k: st[k] for k in ("resident_plans", "peak_bytes", "registered_catalogs", "registered_bytes")},
            "dtype": "f64" if prec else "f32",
            "data": f"synthetic (seeded lognormal surveys, {args.catalogs} catalogs, N_gal log-uniform 1e5-3e6, "
                    f"{args.serve_random_factor:g}x randoms, registered once)",
            "config": {"workload": f"per request: catalog, Nmesh in {sizes}, l_max in {lmaxes} uniform; "
                                   f"L=2500 Mpc/h, TSC + interlacing, dk=0.01; {form.upper()}",
                       "max_inflight": args.inflight, "field_group": args.field_group}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--pipeline", type=int, default=2,
                    help="FP32 estimates in flight in the headline loop, each on its own plan and stream")
    ap.add_argument("--pipeline-fp64", type=int, default=3, help="the same for the FP64 form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ngal", type=int, default=1_000_000)
    ap.add_argument("--random-factor", type=float, default=20.0)
    ap.add_argument("--fp32-only", action="store_true", help="skip the FP64 form (profiling runs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run a plain 1 GiB device copy (x3) first, to calibrate HBM byte counters")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="print the kernel summary of a rocprofv3 CSV output directory and exit")
    ap.add_argument("--cov-mocks", type=int, default=1000, help="mocks of the covariance mode")
    ap.add_argument("--mode", choices=["estimate", "batch", "serve", "basis", "covariance", "fft", "sizes"],
                    default="estimate",
                    help="estimate: the 512^3 l<=4 line (default); batch: covariance mocks; serve: request stream; "
                         "basis: spherical against Cartesian decomposition; covariance: Kaiser-mock wedge "
                         "covariance; fft: the 3D transform against ROCm's FFT library")
    ap.add_argument("--mocks", type=int, default=64)
    ap.add_argument("--plans-per-size", type=int, default=4, help="batch mode: plans (streams) per mesh size")
    ap.add_argument("--requests", type=int, default=2000, help="serve mode: requests of the 0.8 x capacity stream")
    ap.add_argument("--sweep-requests", type=int, default=200, help="serve mode: requests of the other streams")
    ap.add_argument("--burst", type=int, default=100, help="serve mode: requests of the capacity burst")
    ap.add_argument("--load-fractions", type=lambda v: [float(x) for x in v.split(",")], default=[0.8, 0.5, 1.2],
                    help="serve mode: arrival rates as fractions of the measured capacity")
    ap.add_argument("--stream-seconds", type=float, default=None,
                    help="serve mode: cap each stream at about this many seconds of arrivals")
    ap.add_argument("--catalogs", type=int, default=32, help="serve mode: registered catalogs")
    ap.add_argument("--serve-random-factor", type=float, default=10.0)
    ap.add_argument("--serve-precision", type=int, choices=[0, 1], default=0, help="serve mode: 0 FP32, 1 FP64")
    ap.add_argument("--inflight", type=int, default=4)
    ap.add_argument("--field-group", type=int, default=16,
                    help="serve mode: weighted fields per plan group; one plan per mesh size then serves every l_max "
                         "(0: plans sized per request)")
    args = ap.parse_args()
    if args.summarize_profile:
        summarize_profile(args.summarize_profile)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.mode != "estimate":
        out = {"batch": batch_bench, "serve": serve_bench, "basis": basis_bench, "sizes": sizes_bench,
               "covariance": covariance_bench, "fft": fft_bench}[args.mode](args)
        print(json.dumps(out), flush=True)
        return
    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    from synth import config_c2
    t0 = time.perf_counter()
    data, rand, info = config_c2(n_gal=args.ngal, random_factor=args.random_factor)
    log(f"[bench] inputs: {info['n_data']} galaxies, {info['n_rand']} randoms ({time.perf_counter() - t0:.1f} s)")
    kn = math.pi * NMESH / BOX
    edges = np.arange(int(math.floor(kn / 0.01)) + 1, dtype=np.float64) * 0.01
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    gdata = (dev(data.pos), dev(data.w), dev(data.nbar))
    grand = (dev(rand.pos), dev(rand.w), dev(rand.nbar))
    torch.cuda.synchronize()
    upload = catalog_upload(data, rand, gdata + grand)
    res32, sec32, lat32, st32, staged32, one32 = run_form(0, gdata, grand, edges, args.steps, args.warmup,
                                                          args.pipeline)
    log(f"[bench] fp32: {args.steps / sec32:.2f} est/s, {1e3 * sec32 / args.steps:.3f} ms/step with "
        f"{args.pipeline} in flight; one in flight {args.steps / one32:.2f} est/s "
        f"({1e3 * staged32 / args.steps:.3f} ms/step with per-launch events)")
    k64 = args.fp64_steps or args.steps
    if args.fp32_only:
        res64, sec64, lat64, st64, staged64, one64 = res32, float("nan"), np.full(1, np.nan), None, float("nan"), \
            float("nan")
    else:
        res64, sec64, lat64, st64, staged64, one64 = run_form(1, gdata, grand, edges, k64, max(1, args.warmup // 2),
                                                              args.pipeline_fp64)
        log(f"[bench] fp64: {k64 / sec64:.2f} est/s; one in flight {k64 / one64:.2f} est/s")
    ref = golden_poles(info, data, rand) if np.array_equal(edges, np.arange(len(edges)) * 0.01) else None
    vs_oracle = None
    if ref is not None and np.allclose(ref["edges"], edges, rtol=0, atol=1e-12):
        vs_oracle = {"source": "tests/golden/workload_512_l4_poles.txt (FP64 oracle, catalog digest checked)",
                     "tolerance_scaled": {"fp32": 1e-5, "fp64": 1e-12},
                     "fp32": err_vs_oracle(res32, ref)}
        if not args.fp32_only:
            vs_oracle["fp64"] = err_vs_oracle(res64, ref)
        log(f"[bench] vs oracle: {vs_oracle}")
    # FP32 form against the FP64 form (same inputs): the per-bin rule of the parity tests
    raw0 = res64["poles"][0] + res64["shot_noise"]
    scale = np.maximum(np.abs(res64["poles"]), np.abs(raw0)[None, :])
    ok = np.isfinite(res64["poles"])
    fp32_err = float(np.max(np.abs(res32["poles"] - res64["poles"])[ok] / scale[ok]))
    nfields = sum(2 * l + 1 for l in range(2, ELL_MAX + 1, 2))
    n_part = info["n_data"] + info["n_rand"]
    stages = {}
    for name, ms in st32["stage_ms"].items():
        nl = st32["stage_launches"][name]
        if nl == 0 or ms <= 0:
            continue
        b = stage_bytes(NMESH, 4, n_part, nfields)[name] * args.steps
        stages[name] = {"ms_total": round(ms, 3), "launches": nl, "ms_per_launch": round(ms / nl, 4),
                        "algorithmic_GBps": round(b / (ms * 1e-3) / 1e9, 1) if b > 0 else None}
    dom = max(stages, key=lambda k: stages[k]["ms_total"])
    dom_bytes_per_launch = stage_bytes(NMESH, 4, n_part, nfields)[dom] * args.steps / stages[dom]["launches"]
    achieved = dom_bytes_per_launch / (stages[dom]["ms_per_launch"] * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": stored_traffic(dom),
            "bytes_per_launch": dom_bytes_per_launch}
    total_model = sum(stage_bytes(NMESH, 4, n_part, nfields).values())
    out = {
        "metric": METRIC,
        "value": round(args.steps / sec32, 3),
        "unit": "estimates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * sec32 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded lognormal survey mock, resident in HBM)",
        "config": {"workload": "512^3 mesh, L=2500 Mpc/h, TSC + interlacing + compensation, even l <= 4 "
                               "(17 transforms), 64 k bins of 0.01 h/Mpc, 1e6 galaxies + 2e7 randoms",
                   "nmesh": NMESH, "box_len": BOX, "ell_max": ELL_MAX, "n_kbins": len(edges) - 1,
                   "n_data": info["n_data"], "n_rand": info["n_rand"]},
        "latency_ms": {"p50": round(1e3 * float(np.percentile(lat32, 50)), 3),
                       "p99": round(1e3 * float(np.percentile(lat32, 99)), 3)},
        "estimates_in_flight": {"fp32": args.pipeline, "fp64": args.pipeline_fp64},
        "one_in_flight": {"value": round(args.steps / one32, 3), "ms_per_step": round(1e3 * one32 / args.steps, 4)},
        "ms_per_step_with_stage_events": round(1e3 * staged32 / args.steps, 4),
        "err_vs_oracle": vs_oracle,
        "fp64": {"value": round(k64 / sec64, 3), "ms_per_step": round(1e3 * sec64 / k64, 4),
                 "one_in_flight": {"value": round(k64 / one64, 3), "ms_per_step": round(1e3 * one64 / k64, 4)},
                 "stage_ms_per_step": ({k: round(v / k64, 3) for k, v in st64["stage_ms"].items() if v > 0}
                                       if not args.fp32_only else None),
                 "latency_ms": {"p50": round(1e3 * float(np.percentile(lat64, 50)), 3),
                                "p99": round(1e3 * float(np.percentile(lat64, 99)), 3)}},
        "fp32_vs_fp64_max_scaled_err": fp32_err,
        "catalog_upload": dict(upload, estimates_per_s_incl_pinned_upload=round(
            1.0 / (sec32 / args.steps + 1e-3 * upload["ms_pinned"]), 3)),
        "model_GB_per_estimate_fp32": round(total_model / 1e9, 3),
        "effective_GBps_fp32": round(total_model * args.steps / sec32 / 1e9, 1),
        "roofline": roof,
        "stages": stages,
    }
    if not args.no_cpu_baseline:
        workers = max(1, min(16, os.cpu_count() or 1))
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(data, rand, edges, workers)
        log(f"[bench] cpu baseline sample took {time.perf_counter() - t0:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
