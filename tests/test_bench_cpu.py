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
