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


def test_sort_bytes_follow_element_formats():
    n = 1 << 24
    assert bench.sort_forms(n, 8) == ["key64", "key64", "key64", "pack64", "pack64", "pack64",
                                      "pack64", "pack32", "idx"]
    b8 = bench.kernel_bytes(n, 0, 0, 8, "fp64")["sort_pass"] / n
    # pass 0 reads the key alone; key + index (12) until 40 key bits (the
    # leading 1 included) + 24 index bits fit in 8 bytes; 8 + 24 bits fit in 4;
    # the last pass writes the index
    assert b8 == (8 + 12) + (12 + 12) + (12 + 8) + 3 * (8 + 8) + (8 + 4) + (4 + 4)
    # 2^26 elements: 40 + 26 bits do not fit in 64, 8 + 26 not in 32
    assert bench.sort_forms(1 << 26, 8) == ["key64"] * 4 + ["pack64"] * 4 + ["idx"]
    # 9-bit digits: 37 + 24 bits fit after the third pass; 10 + 24 never fit in 32
    assert bench.sort_forms(1 << 24, 9) == ["key64"] * 3 + ["pack64"] * 4 + ["idx"]


def test_batch_set_index_bits_pack_earlier():
    # 1.6e8 particles need 28 index bits; sets of at most 2^18 need 18
    n = 159_638_865
    assert bench.sort_forms(n, 8) == ["key64"] * 4 + ["pack64"] * 4 + ["idx"]
    assert bench.sort_forms(n, 8, 18) == ["key64"] * 3 + ["pack64"] * 4 + ["pack32", "idx"]
    assert bench.sort_forms(n, 8, 30) == bench.sort_forms(n, 8)  # a looser bound changes nothing
    full = bench.kernel_bytes(n, 0, 0, 8, "fp64")["sort_pass"] / n
    tight = bench.kernel_bytes(n, 0, 0, 8, "fp64", 18)["sort_pass"] / n
    assert (full, tight) == (148, 132)


SUPPORTED_PAIRS = {("key64", "key64"), ("key64", "pack64"), ("pack64", "pack64"),
                   ("pack64", "pack32"), ("pack64", "idx"), ("pack32", "pack32"),
                   ("pack32", "idx")}


def test_sort_form_pairs_are_the_instantiated_ones():
    """Every (read, write) pair the plan can produce for 8- and 9-bit digits is
    one the radix pass is built for."""
    sizes = {1, 2, 3}
    for b in range(1, 32):
        sizes |= {(1 << b) - 1, 1 << b, (1 << b) + 1}
    for bits in (8, 9):
        for n in sorted(sizes):
            f = bench.sort_forms(n, bits)
            for pair in zip(f[:-1], f[1:]):
                assert pair in SUPPORTED_PAIRS, (n, bits, f)


def _emulate_packed_sort(keys, bits, ib):
    """The radix passes as the kernels compute them: digit at bit k*bits of a
    64-bit key or at bit ib of a packed word; a packed word is written as
    (word >> (shift + bits)) << ib | index, truncated to its width.  Every
    pass's digit must be the key's digit k (what the key kernel counted for the
    global digit offsets)."""
    n = keys.shape[0]
    forms = bench.sort_forms(1 << ib, bits)
    mask = np.uint64((1 << ib) - 1)
    dmask = np.uint64((1 << bits) - 1)
    words, idx = keys.copy(), np.arange(n, dtype=np.uint64)
    for k in range(len(forms) - 1):
        fi, fo = forms[k], forms[k + 1]
        shift = k * bits if fi == "key64" else ib
        if fi != "key64":
            idx = words & mask
        d = (words >> np.uint64(shift)) & dmask
        assert np.array_equal(d, (keys[idx.astype(np.int64)] >> np.uint64(k * bits)) & dmask), \
            (k, fi)
        order = np.argsort(d, kind="stable")
        words, idx = words[order], idx[order]
        if fo in ("pack64", "pack32"):
            words = ((words >> np.uint64(shift + bits)) << np.uint64(ib)) | idx
            if fo == "pack32":
                words &= np.uint64(0xFFFFFFFF)
    return idx


@pytest.mark.parametrize("bits", [8, 9])
@pytest.mark.parametrize("ib", [1, 2, 7, 12, 23, 24, 25, 26, 28, 31])
def test_packed_passes_sort_stably(bits, ib):
    rng = np.random.default_rng(ib * 10 + bits)
    n = min(4000, 1 << ib)  # the indices fit in ib bits
    body = rng.integers(0, 1 << 63, n, dtype=np.uint64)
    # duplicates and keys that differ only in the lowest or highest bits
    body[::7] = body[1::7][: body[::7].shape[0]]
    body[3::11] ^= np.uint64(1)
    body[5::13] ^= np.uint64(1 << 62)
    keys = body | np.uint64(1 << 63)
    got = _emulate_packed_sort(keys, bits, ib)
    want = np.argsort(keys, kind="stable")
    assert np.array_equal(got, want.astype(np.uint64))


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


def test_source_hash_ignores_comments_only():
    src = 'int a = 1; // note\n/* block\n comment */ char s[] = "//x /*y*/";\n\n  int b;  \n'
    assert bench.code_text(src) == 'int a = 1;\n  char s[] = "//x /*y*/";\n  int b;'
    same = src.replace("// note", "// another note").replace("block", "other")
    assert bench.code_text(same) == bench.code_text(src)
    assert bench.code_text(src.replace("int b;", "int c;")) != bench.code_text(src)


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
# the per-set radix tiles and key chunks of a batch, emulated on the CPU
# --------------------------------------------------------------------------
# A batch sorts every set in place (tb_keys.hip k_setup / k_tile_map /
# k_keygen_sets; tb_sort.hip k_onesweep):
#   tiles  : set b has ceil(n_b / TILE) radix tiles starting at tile_start[b]
#            (an exclusive scan over the sets), tile_set[t] = last b with
#            tile_start[b] <= t; tile t of set b holds positions
#            [off[b] + (t - tile_start[b]) TILE, min(+TILE, off[b + 1]));
#   chunks : the same with kBboxChunk = 65536 for the key kernel's chunks;
#   grid   : one workgroup per possible tile, N / TILE + B + ... of them; those
#            past tile_start[B] leave at once.
# The emulation checks that the tiles and chunks of every layout cover each
# set exactly once, never straddle a set, and that every index stays inside
# the tables and the workspace the plan sizes.

TILE = 512 * 11
CHUNK = 65536


def _random_layout(rng):
    nsets = int(rng.choice([2, 7, 64, 1000, 4096, 16383]))
    sizes = rng.integers(0, rng.choice([3, 40, 3000, 70000]), nsets)
    sizes[rng.random(nsets) < 0.2] = 0  # empty sets anywhere, also at both ends
    if sizes.sum() == 0:
        sizes[rng.integers(0, nsets)] = 1
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return nsets, off


def _tables(off, unit):
    sizes = np.diff(off)
    per = (sizes + unit - 1) // unit
    start = np.concatenate([[0], np.cumsum(per)]).astype(np.int64)
    t = np.arange(start[-1], dtype=np.int64)
    owner = np.searchsorted(start, t, side="right") - 1  # last b with start[b] <= t
    lo = off[owner] + (t - start[owner]) * unit
    hi = np.minimum(lo + unit, off[owner + 1])
    return start, owner, lo, hi


def test_batch_tiles_and_chunks_emulation():
    rng = np.random.default_rng(2024)
    checked = 0
    for _ in range(300):
        nsets, off = _random_layout(rng)
        n = int(off[-1])
        for unit, bound in ((TILE, (n + TILE - 1) // TILE + nsets),
                            (CHUNK, (n + CHUNK - 1) // CHUNK + nsets)):
            start, owner, lo, hi = _tables(off, unit)
            assert start[-1] <= bound  # the plan's grid and table sizes
            assert np.all((owner >= 0) & (owner < nsets))
            assert np.all(lo < hi) and np.all(hi - lo <= unit)
            assert np.all((off[owner] <= lo) & (hi <= off[owner + 1]))  # never straddles a set
            # every position exactly once: within a set the tiles abut, a set's
            # first tile starts at its first position and its last ends at its end
            same = owner[1:] == owner[:-1]
            assert np.all(lo[1:][same] == hi[:-1][same])
            assert np.all(hi[:-1][~same] == off[owner[:-1][~same] + 1])
            sizes = np.diff(off)
            assert np.array_equal(np.bincount(owner, weights=hi - lo, minlength=nsets), sizes)
            # a set's first tile starts its look-back chain: tile == start[owner]
            first = np.arange(start[-1]) == start[owner]
            assert np.array_equal(lo[first], off[owner[first]])
            checked += len(lo)
    assert checked > 100_000
