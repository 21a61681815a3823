"""Parity at the full benchmark sizes, in the launch configurations bench.py
times: structure checked through properties that determine the tree uniquely,
moments on sampled cells (or whole sampled sets) against the oracle.

  mixed16m      N = 2^24 clustered, log-normal masses, n_leaf 8, TB_MIXED
  batched4096   4,096 Plummer sets (about 1.6e8 particles), n_leaf 16, one
                graph-captured batch
  clustered64m  N = 2^26 clustered, n_leaf 8, FP64
"""
import numpy as np
import pytest
import torch

import oracle
import treecheck as tc
from paper_2312_06102_amd import autotune
from paper_2312_06102_amd import datagen as dg
from paper_2312_06102_amd import treebuild as tb
from test_gpu_batched import check_against_oracle, set_view
from test_gpu_parity import FP64_TOL, MIXED_TOL, compare_structure, moment_errors

pytestmark = pytest.mark.gpu


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _np(res):
    out = {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in res.items()}
    out["cell_key"] = out["cell_key"].view(np.uint64)
    if "key_sorted" in out:
        out["key_sorted"] = out["key_sorted"].view(np.uint64)
    return out


def sampled_moments(pos, mass, g, tol, n_sample=300, seed=99, max_count=1 << 22):
    rng = _rng(seed)
    C = g["n_cells"]
    sample = np.unique(np.concatenate([[0, 1, 2], rng.integers(0, C, n_sample),
                                       np.asarray(g["level_offset"][:21]).clip(max=C - 1)]))
    worst = np.zeros(3)
    for c in sample:
        f, k = int(g["cell_first"][c]), int(g["cell_count"][c])
        if k > max_count and c != 0:
            continue
        lvl = int(g["cell_level"][c])
        oc, oq = oracle.cell_moments(pos, mass, g["perm"], f, k, int(g["cell_key"][c]), lvl)
        e = moment_errors(g["com"][c:c + 1].astype(np.float64), g["quad"][c:c + 1].astype(np.float64),
                          oc[None], oq[None], np.array([lvl]))
        worst = np.maximum(worst, e)
        assert max(e) <= tol, (c, e)
    return worst


def structure_checks(pos, g, nl):
    n = pos.shape[0]
    _, keys = oracle.keys(pos)
    perm = g["perm"].astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(n))
    sk = keys[perm]
    assert np.all(sk[1:] >= sk[:-1])
    ties = sk[1:] == sk[:-1]
    assert np.all(perm[1:][ties] > perm[:-1][ties])
    tc.check_invariants(g, sk, nl)
    return sk


@pytest.mark.timeout(1200)
def test_full_size_mixed16m():
    """Mixed precision at N = 2^24 (clustered, log-normal masses): the tree bit
    for bit against a full oracle build and against the FP64 GPU path on the same
    data; the FP32 + Kahan moments of every cell within 1e-6 of the FP64 oracle."""
    import time
    pos, mass, nl = dg.workload("mixed16m")
    print("[full mixed] generated", flush=True)
    p = torch.from_numpy(pos).cuda()
    m = torch.from_numpy(mass).cuda()
    b = tb.Builder(pos.shape[0], nl, "mixed")
    b.launch(p, m, ((0.0, 0.0, 0.0), 1.0))
    g = _np(b.result())
    ref = _np(tb.build(p, m, nl, ((0.0, 0.0, 0.0), 1.0)))  # FP64 path, same data
    del p, m
    print(f"[full mixed] built, {g['n_cells']} cells", flush=True)
    # the tree does not depend on the moment precision
    compare_structure(g, ref)
    t0 = time.time()
    o = oracle.build(pos, mass, nl)
    print(f"[full mixed] oracle built in {time.time() - t0:.1f} s", flush=True)
    compare_structure(g, o)
    e32 = moment_errors(g["com"].astype(np.float64), g["quad"].astype(np.float64), o["com"],
                        o["quad"], o["cell_level"])
    e64 = moment_errors(ref["com"], ref["quad"], o["com"], o["quad"], o["cell_level"])
    print(f"[full mixed] all cells, mixed vs oracle M={e32[0]:.2e} com={e32[1]:.2e} "
          f"Q={e32[2]:.2e}; FP64 vs oracle M={e64[0]:.2e} com={e64[1]:.2e} Q={e64[2]:.2e}",
          flush=True)
    assert max(e32) <= MIXED_TOL, e32
    assert max(e64) <= FP64_TOL, e64


def test_full_size_batched4096_graph():
    sizes = dg.batched_sizes(4096, 256, 262144, seed=4)
    pos, mass, offsets = dg.batched_plummer(sizes, seed=4)
    N, B = pos.shape[0], len(sizes)
    print(f"[full batch] generated N={N}", flush=True)
    p = torch.from_numpy(pos).cuda()
    m = torch.from_numpy(mass).cuda()
    off = torch.from_numpy(offsets).cuda()
    boxes = torch.tensor([[0.0, 0.0, 0.0, 1.0]] * B, dtype=torch.float64, device="cuda")
    # the configuration the benchmark times: the autotuner's sort shape and the
    # set-size bound of the largest set
    set_bits = max(1, (int(sizes.max()) - 1).bit_length())
    k = autotune.tune(p, m, 16, "fp64", set_offsets=off, boxes=boxes, use_cache=False,
                      set_index_bits=set_bits)
    print(f"[full batch] sort config {k}, set index bits {set_bits}", flush=True)
    bb = tb.BatchBuilder(N, B, 16, "fp64", k, sorted_keys=True, set_index_bits=set_bits)
    bb.capture(p, m, off, boxes)
    bb.replay()
    bb.replay()
    res = bb.result()
    # bit-identical to the default shape without the bound
    ref = tb.build_batched(p, m, off, 16, boxes, sorted_keys=True)
    for name in ("perm", "cell_key", "cell_level", "cell_first", "cell_count", "child_ptr",
                 "com", "quad", "level_offset", "cell_offsets", "key_sorted"):
        assert torch.equal(res[name], ref[name]), name
    assert res["n_cells"] == ref["n_cells"]
    del ref
    g = _np(res)
    print(f"[full batch] built, {g['n_cells']} cells, equal to the unbounded default", flush=True)
    co = g["cell_offsets"]
    assert co[0] == 0 and co[-1] == g["n_cells"] and np.all(np.diff(co) > 0)
    assert np.array_equal(g["level_offset"][:, 0], co[:-1])
    assert np.array_equal(g["level_offset"][:, -1], co[1:])
    # every set's permutation stays inside its own range, keys sorted per set
    sp = g["perm"].astype(np.int64)
    set_of = np.repeat(np.arange(B), sizes)
    assert np.array_equal(set_of[sp], set_of)
    ks = g["key_sorted"]
    inner = np.ones(N - 1, bool)
    inner[offsets[1:-1] - 1] = False
    assert np.all(ks[1:][inner] >= ks[:-1][inner])
    print("[full batch] permutation ok", flush=True)
    # whole sets against the oracle: smallest, largest and a random sample
    rng = _rng(7)
    sets = np.unique(np.concatenate([[int(np.argmin(sizes)), int(np.argmax(sizes)), 0, B - 1],
                                     rng.integers(0, B, 24)]))
    worst = check_against_oracle(pos, mass, offsets, 16, g, sets)
    print(f"[full batch] {len(sets)} sets vs oracle, max rel err {worst}", flush=True)


def test_full_size_clustered64m():
    pos, mass, nl = dg.workload("clustered64m")
    print("[full clustered] generated", flush=True)
    p = torch.from_numpy(pos).cuda()
    m = torch.from_numpy(mass).cuda()
    g = _np(tb.build(p, m, nl, ((0.0, 0.0, 0.0), 1.0)))
    del p, m
    print(f"[full clustered] built, {g['n_cells']} cells", flush=True)
    structure_checks(pos, g, nl)
    print("[full clustered] invariants ok", flush=True)
    sampled_moments(pos, mass, g, FP64_TOL)


def test_counted_passes_at_full_size():
    """N = 2^24 with a 4096-key sort tile (exactly 4096 tiles): the counted
    passes (the default) must give a tree bit-identical to the look-back build,
    and the perm must sort the keys stably."""
    cfgs = tb.tb_sort_configs()
    k = next(i for i, (bits, ipt, thr) in enumerate(cfgs) if bits == 8 and ipt * thr == 4096)
    pos, mass = dg.plummer(1 << 24, seed=2)
    p, m = torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda()
    box = ((0.0, 0.0, 0.0), 1.0)
    print(f"[fullsize] plummer 2^24 sort_config {k} {cfgs[k]} counted vs look-back", flush=True)
    a = _np(tb.build(p, m, 16, box, sort_config=k))
    b = _np(tb.build(p, m, 16, box, sort_config=k, lookback=True))
    compare_structure(a, b)
    assert np.array_equal(a["com"], b["com"]) and np.array_equal(a["quad"], b["quad"])
    structure_checks(pos, a, 16)
