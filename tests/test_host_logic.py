"""Host-side logic that needs no GPU: the autotuner's cache, the benchmark's
byte models and its guard on stale counter profiles, the one-GPU contract."""
import json
import os
import subprocess
import sys

import numpy as np
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


# --------------------------------------------------------------------------
# the batched set lookup through the coarse set table, emulated on the CPU
# --------------------------------------------------------------------------
# The key kernel and the set-id sort passes find the set that holds position x
# as follows (tb_keys.hip, k_setup / k_keygen; tb_sort.hip, k_onesweep):
#   shift  : smallest s with ceil(n / 2^s) <= K_COARSE                (make_plan)
#   coarse : coarse[k] = last b with off[b] <= min(k << shift, n - 1),
#            for k = 0 .. ((n - 1) >> shift)                            (k_setup)
#   lookup : k = x >> shift; b = last index in [coarse[k], coarse[k + 1]]
#            with off[b] <= x, found by the kernels' binary search; the key
#            kernel clamps x to n - 1 for lanes past the end and b to B - 1.
# The emulation checks that every index stays inside the table and that the
# set found is the one a plain search over all offsets finds.

K_COARSE = 4096


def _coarse_shift(n):
    s = 0
    while (n + (1 << s) - 1) >> s > K_COARSE:
        s += 1
    return s


def _upper_index_in(tab, lo, hi, x):
    """Vectorised copy of the kernels' search: last b in [lo, hi] with tab[b] <= x,
    given tab[lo] <= x."""
    lo, hi = lo.copy(), hi.copy()
    while True:
        act = lo < hi
        if not act.any():
            return lo
        mid = (lo + hi + 1) >> 1
        ok = tab[np.minimum(mid, len(tab) - 1)] <= x
        lo = np.where(act & ok, mid, lo)
        hi = np.where(act & ~ok, mid - 1, hi)


def _random_layout(rng):
    nsets = int(rng.choice([1, 2, 7, 64, 1000, 4096, 16383]))
    sizes = rng.integers(0, rng.choice([3, 40, 3000, 70000]), nsets)
    sizes[rng.random(nsets) < 0.2] = 0  # empty sets anywhere, also at both ends
    if sizes.sum() == 0:
        sizes[rng.integers(0, nsets)] = 1
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return nsets, off


def test_coarse_set_lookup_emulation():
    rng = np.random.default_rng(2024)
    lookups = 0
    for _ in range(300):
        nsets, off = _random_layout(rng)
        n = int(off[-1])
        shift = _coarse_shift(n)
        K = ((n - 1) >> shift) + 1
        assert K <= K_COARSE
        kpos = np.minimum(np.arange(K + 1, dtype=np.int64) << shift, n - 1)
        # k_setup: the set holding each coarse position (search over all B + 1 offsets)
        coarse = _upper_index_in(off, np.zeros(K + 1, np.int64), np.full(K + 1, nsets, np.int64),
                                 kpos)
        assert coarse.max() <= nsets - 1  # off[B] = n is never <= a position below n
        # every position of small batches, a sample plus every set boundary of large
        # ones, and lanes past the end (clamped to n - 1 by the key kernel)
        if n <= 20000:
            x = np.arange(n, dtype=np.int64)
        else:
            edges = np.concatenate([off[:-1], off[1:] - 1, kpos]).clip(0, n - 1)
            x = np.concatenate([rng.integers(0, n, 20000), edges])
        x = np.concatenate([x, np.full(64, n - 1, np.int64)])
        k = x >> shift
        assert k.max() + 1 <= K  # both table entries read stay inside the K + 1 entries
        lo, hi = coarse[k], coarse[k + 1]
        assert np.all(off[lo] <= x) and np.all(lo <= hi)
        b = np.minimum(_upper_index_in(off, lo, hi, x), nsets - 1)
        want = np.searchsorted(off, x, side="right") - 1
        assert np.array_equal(b, want)
        assert np.all((off[b] <= x) & (x < off[b + 1]))  # a non-empty set holding x
        lookups += x.size
    assert lookups > 5_000_000
