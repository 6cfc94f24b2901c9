"""CPU tests of bench.py's host logic: the one-GPU guard, the stored HBM traffic that the
roofline reports (keyed by the digest of the transform kernels' sources), the algorithmic
bytes it is compared with, and the rocprofv3 CSV summary."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""   # no JSON line


def _fake_tree(tmp_path, monkeypatch, content: str):
    monkeypatch.setattr(bench, "HERE", str(tmp_path))
    for rel in bench.TRAFFIC_SOURCES:
        p = tmp_path / rel
        p.parent.mkdir(parents=True, exist_ok=True)
        p.write_text(content)
    (tmp_path / "profiles").mkdir(exist_ok=True)


def test_stored_traffic_follows_the_source_digest(tmp_path, monkeypatch):
    _fake_tree(tmp_path, monkeypatch, "kernel sources, first version\n")
    dig = bench.source_digest()
    recs = [dict(stage="xpost", nmesh=bench.NMESH, hbm_bytes_per_launch=123, source_digest=dig),
            dict(stage="zpre", nmesh=bench.NMESH, hbm_bytes_per_launch=456, source_digest="0" * 16),
            dict(stage="ycol", nmesh=256, hbm_bytes_per_launch=789, source_digest=dig)]
    (tmp_path / "profiles" / "k_traffic.txt").write_text(
        "# header\n" + "".join("TRAFFIC " + json.dumps(r) + "\n" for r in recs))
    assert bench.stored_traffic("xpost") == 123
    assert bench.stored_traffic("zpre") is None      # taken from other sources
    assert bench.stored_traffic("ycol") is None      # another mesh size
    assert bench.stored_traffic("xcombine") is None  # never measured
    # any edit of a listed source (comments included) retires the stored reading
    (tmp_path / bench.TRAFFIC_SOURCES[-1]).write_text("kernel sources, second version\n")
    assert bench.source_digest() != dig
    assert bench.stored_traffic("xpost") is None


def test_committed_traffic_records_use_the_bench_algorithmic_bytes():
    """Every committed TRAFFIC record states the algorithmic bytes that bench.py divides by
    the kernel time (one read and one write of every element a pass touches)."""
    recs = []
    for name in sorted(os.listdir(os.path.join(ROOT, "profiles"))):
        if name.endswith("_traffic.txt"):
            with open(os.path.join(ROOT, "profiles", name)) as f:
                recs += [json.loads(l[len("TRAFFIC "):]) for l in f if l.startswith("TRAFFIC ")]
    assert recs, "no stored traffic records"
    nfields = 14   # l <= 4: 5 + 9 weighted fields
    for r in recs:
        es = 4 if r["precision"] == "fp32" else 8
        want = bench.stage_bytes(r["nmesh"], es, 0, nfields)[r["stage"]]
        if r["stage"] == "ycol":
            want /= 2  # two launches per estimate: the record is the mean per launch
        assert r["algorithmic_bytes_per_launch"] == pytest.approx(want, rel=1e-12), r["stage"]
        assert 0.9 < r["hbm_bytes_per_launch"] / r["algorithmic_bytes_per_launch"] < 2.0, r["stage"]


def test_summarize_profile_reads_stats_and_counters(tmp_path, capsys):
    d = tmp_path / "prof"
    d.mkdir()
    (d / "run_kernel_stats.csv").write_text(
        "Name,Calls,TotalDurationNs,AverageNs,Percentage\n"
        '"void pkm::(anonymous namespace)::k_xpost<float, 8, 512, 4, false>(int, int)",6,22000000,3666666.7,60.0\n'
        '"pkm::k_reduce(double const*, int)",6,48000,8000,0.1\n')
    (d / "run_counter_collection.csv").write_text(
        "Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n"
        '1,"pkm::k_zfwd<float, 8, 512, 8>(int)",FETCH_SIZE,100\n'
        '1,"pkm::k_zfwd<float, 8, 512, 8>(int)",FETCH_SIZE,50\n'
        '2,"pkm::k_zfwd<float, 8, 512, 8>(int)",FETCH_SIZE,150\n')
    bench.summarize_profile(str(d))
    out = capsys.readouterr().out.splitlines()
    xp = [l for l in out if l.startswith("k_xpost<float, 8, 512, 4, false>")]
    assert len(xp) == 1 and xp[0].split()[-4:] == ["6", "3666.7", "22.000", "60.00"]
    zf = [l for l in out if l.startswith("k_zfwd<float, 8, 512, 8>")]
    # counter rows of one dispatch (one per XCD or shader engine) add up; the mean is per dispatch
    assert len(zf) == 1 and zf[0].split()[-3:] == ["FETCH_SIZE", "2", "150"]


def test_err_vs_oracle_and_golden_guard(tmp_path, monkeypatch):
    """The bench line's error against the stored FP64 oracle: the scaled per-bin rule of the
    parity tests, and no comparison at all when the stored catalog does not match the run."""
    import numpy as np
    from synth import Catalog
    po = np.array([[10.0, 20.0, 30.0], [1.0, -2.0, 0.5], [0.1, 0.2, -0.3]])
    ref = {"poles": po, "n_modes": np.array([4, 8, 12]), "shot_noise": 5.0}
    res = {"poles": po + np.array([[1e-4, 0, 0], [0, 3e-4, 0], [0, 0, 0]]), "n_modes": np.array([4, 8, 12])}
    e = bench.err_vs_oracle(res, ref)
    # l=0 bin 0: 1e-4 / max(10, 15); l=2 bin 1: 3e-4 / max(2, 25)
    assert abs(e["max_scaled"] - 3e-4 / 25.0) < 1e-15 and e["n_modes_equal"]
    assert abs(e["max_plain_rel"] - 1.5e-4) < 1e-12
    # a stored file for other inputs is ignored
    monkeypatch.setattr(bench, "HERE", str(tmp_path))
    (tmp_path / "tests" / "golden").mkdir(parents=True)
    cat = Catalog(np.zeros((2, 3)), np.ones(2), np.ones(2))
    (tmp_path / "tests" / "golden" / "workload_512_l4_poles.txt").write_text(
        "# catalog: synth.config_c2(), n_data 2, n_rand 2, digest ffffffffffffffff\n# shot_noise 1.0\n"
        "0.0 0.01 4 0.005 1.0 2.0 3.0\n")
    assert bench.golden_poles({"n_data": 2, "n_rand": 2}, cat, cat) is None
    assert bench.golden_poles({"n_data": 3, "n_rand": 2}, cat, cat) is None
    from synth import catalog_digest
    (tmp_path / "tests" / "golden" / "workload_512_l4_poles.txt").write_text(
        f"# catalog: synth.config_c2(), n_data 2, n_rand 2, digest {catalog_digest(cat, cat)}\n# shot_noise 1.0\n"
        "0.0 0.01 4 0.005 1.0 2.0 3.0\n")
    g = bench.golden_poles({"n_data": 2, "n_rand": 2}, cat, cat)
    assert g is not None and g["poles"].shape == (3, 1) and g["n_modes"][0] == 4


class _FakePlan:
    """Stands in for a plan: records the order of enqueue and finish calls."""

    def __init__(self, name, log):
        self.name, self.log, self.pending = name, log, []

    def enqueue(self, data, rand):
        assert not self.pending, f"{self.name}: enqueue while an estimate is in flight"
        self.log.append(("enqueue", self.name))
        self.pending.append(len([e for e in self.log if e[0] == "enqueue"]) - 1)

    def finish(self):
        assert self.pending, f"{self.name}: finish without an estimate"
        self.log.append(("finish", self.name))
        return self.pending.pop()


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("steps", [1, 2, 5, 20])
def test_in_flight_loop_finishes_every_estimate(k, steps):
    log = []
    plans = [_FakePlan(i, log) for i in range(k)]
    res, done = bench.run_in_flight(plans, steps, None, None)
    assert done == steps
    enq = [p for op, p in log if op == "enqueue"]
    fin = [p for op, p in log if op == "finish"]
    assert enq == [i % k for i in range(steps)]          # estimate i on plan i mod k
    assert sorted(fin) == sorted(enq)                    # every estimate finished
    assert all(not p.pending for p in plans)
    assert res == steps - 1                              # the last estimate enqueued is finished last
    # at most k estimates in flight at any time
    inflight = peak = 0
    for op, _ in log:
        inflight += 1 if op == "enqueue" else -1
        peak = max(peak, inflight)
    assert peak == min(k, steps)
