"""Host-side logic that needs no GPU: the autotuner's cache, the benchmark's
byte models and its guard on stale counter profiles, the one-GPU contract."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2312_06102_amd import autotune  # noqa: E402


def test_autotune_cache_roundtrip(tmp_path):
    path = str(tmp_path / "tune.json")
    assert autotune.lookup(1 << 24, 1, 16, "fp64", path=path) is None
    key = autotune.size_class(1 << 24, 1, 16, "fp64")
    autotune._store(path, key, {"sort_config": 3, "shape": [8, 16, 256], "ms": {"3": 1.0}})
    assert autotune.lookup(1 << 24, 1, 16, "fp64", path=path) == 3
    # the size class rounds log2 of N and of the set count
    assert autotune.lookup(int(1.2 * (1 << 24)), 1, 16, "fp64", path=path) == 3
    assert autotune.lookup(1 << 26, 1, 16, "fp64", path=path) is None
    assert autotune.lookup(1 << 24, 4096, 16, "fp64", path=path) is None
    assert autotune.lookup(1 << 24, 1, 16, "mixed", path=path) is None
    # a second entry keeps the first
    autotune._store(path, autotune.size_class(1 << 20, 1, 8, "fp64"), {"sort_config": 1})
    data = json.load(open(path))
    assert len(data) == 2


def test_autotune_cache_tolerates_damage(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert autotune.lookup(1000, 1, 16, path=str(path)) is None


def test_sort_bytes_follow_key_widths():
    n = 1 << 20
    b8 = bench.kernel_bytes(n, 0, 0, 8, 0, "fp64")["sort_pass"] / n
    # passes 0..3 read 64-bit keys (pass 3 writes their upper halves), passes
    # 4..6 move 32-bit keys, the last writes no key; payload 4 B in and out
    assert b8 == (8 + 0 + 8 + 4) + 2 * (8 + 4 + 8 + 4) + (8 + 4 + 4 + 4) + 2 * (4 + 4 + 4 + 4) \
        + (4 + 4 + 4 + 4) + (4 + 4 + 0 + 4)
    b9 = bench.kernel_bytes(n, 0, 0, 7, 0, "fp64")["sort_pass"] / n
    assert b9 == (8 + 0 + 8 + 4) + 2 * (8 + 4 + 8 + 4) + (8 + 4 + 4 + 4) + 2 * (4 + 4 + 4 + 4) \
        + (4 + 4 + 0 + 4)


def test_method_bytes_model():
    n, cells = 1 << 24, 4_000_000
    c = cells / n
    assert bench.method_bytes(n, cells, 8, "fp64") == pytest.approx(n * (56 + 24 * 8 + 185 * c))
    assert bench.method_bytes(n, cells, 8, "mixed") == pytest.approx(n * (56 + 24 * 8 + 105 * c))


def test_counter_profile_is_ignored_once_sources_change(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    prof = {"file": "x", "source_sha256": bench.source_hash(),
            "kernels": {"sort_pass": {"bytes_per_launch": 1e8, "launches_per_build": 8}}}
    (tmp_path / "pmc_w.json").write_text(json.dumps(prof))
    assert bench.counter_traffic("w") is not None
    assert bench.counter_summary("w", 1.0)["bytes_per_build"] == 8e8
    prof["source_sha256"] = "0" * 64
    (tmp_path / "pmc_w.json").write_text(json.dumps(prof))
    assert bench.counter_traffic("w") is None
    assert bench.counter_traffic("missing") is None


def test_committed_counter_profiles_are_well_formed():
    pdir = os.path.join(ROOT, "profiles")
    for f in os.listdir(pdir):
        if f.startswith("pmc_") and f.endswith(".json"):
            prof = json.load(open(os.path.join(pdir, f)))
            assert len(prof["source_sha256"]) == 64
            assert prof["calibration"]["fetch_scale"] > 0 and prof["calibration"]["write_scale"] > 0
            for st, k in prof["kernels"].items():
                assert k["bytes_per_launch"] == pytest.approx(
                    k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"])
                assert k["launches_per_build"] > 0


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]
