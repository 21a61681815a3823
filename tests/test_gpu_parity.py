"""HIP path vs the CPU oracle, element by element, through the C ABI.

Structure (perm, keys, cells, links, level offsets) must be bit-identical.
FP64 moments must agree to 1e-12 in the per-cell relative measures
  e_M = |dM| / M,  e_com = max|d com| / l,  e_Q = max|d Q| / (M l^2),
with l = side * 2^-depth (the cell side).  Moments are unique up to rounding;
the normalisation by the cell's own size keeps single-particle leaves (Q = 0)
and deep cells comparable.
"""
import numpy as np
import pytest
import torch

import oracle
import treecheck as tc
from paper_2312_06102_amd import datagen as dg
from paper_2312_06102_amd import treebuild as tb

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def gpu_build(pos, mass, n_leaf, box=((0.0, 0.0, 0.0), 1.0), **kw):
    print(f"[gpu_build] N={pos.shape[0]} n_leaf={n_leaf} box={box} {kw}", flush=True)
    p = torch.from_numpy(np.ascontiguousarray(pos, np.float32)).cuda()
    m = torch.from_numpy(np.ascontiguousarray(mass, np.float32)).cuda()
    res = tb.build(p, m, n_leaf, box, sorted_keys=True, **kw)
    out = {}
    for k, v in res.items():
        out[k] = v.cpu().numpy() if torch.is_tensor(v) else v
    out["cell_key"] = out["cell_key"].view(np.uint64)
    out["key_sorted"] = out["key_sorted"].view(np.uint64)
    return out


def compare_structure(g, o):
    assert g["n_cells"] == o["n_cells"]
    assert np.array_equal(g["perm"], o["perm"])
    assert np.array_equal(g["cell_key"], o["cell_key"])
    assert np.array_equal(g["cell_level"], o["cell_level"])
    assert np.array_equal(g["cell_first"], o["cell_first"])
    assert np.array_equal(g["cell_count"], o["cell_count"])
    assert np.array_equal(g["child_ptr"], o["child_ptr"])
    assert np.array_equal(g["level_offset"], o["level_offset"])


def moment_errors(g_com, g_quad, o_com, o_quad, level, side=1.0, extent=None):
    """Max relative errors.  `extent` (optional, per cell) replaces the cell side
    when particles lie outside their cell (points outside the root box are
    clamped into edge cells for the key but keep their true positions)."""
    l = side * np.ldexp(1.0, -level.astype(np.int64))
    if extent is not None:
        l = np.maximum(l, extent)
    M = o_com[:, 3]
    e_m = np.abs(g_com[:, 3] - M) / M
    e_c = np.max(np.abs(g_com[:, :3] - o_com[:, :3]), axis=1) / l
    e_q = np.max(np.abs(g_quad - o_quad), axis=1) / (M * l * l)
    return e_m.max(initial=0), e_c.max(initial=0), e_q.max(initial=0)


def cell_extents(pos, o, lo=(0.0, 0.0, 0.0), side=1.0, curve="morton"):
    """Side of the smallest cube about each cell centre that holds its particles."""
    ext = np.zeros(o["n_cells"])
    u = pos.astype(np.float64) - np.asarray(lo, np.float64)
    for c in range(o["n_cells"]):
        f, k = int(o["cell_first"][c]), int(o["cell_count"][c])
        key, d = int(o["cell_key"][c]), int(o["cell_level"][c])
        if curve == "hilbert":
            ijk = oracle.hilbert_decode(np.array([key & ((1 << (3 * d)) - 1)], np.uint64), d)[0]
            off = (ijk.astype(np.float64) + 0.5) * side * 2.0 ** -d
        else:
            off = np.array([float(v) for v in tc.cell_centre_offset(key, d, side)])
        ext[c] = 2.0 * np.abs(u[o["perm"][f:f + k]] - off).max()
    return ext


def full_parity(pos, mass, n_leaf, lo=(0.0, 0.0, 0.0), side=1.0, box="given", extent=False, **kw):
    curve = kw.get("curve", "morton")
    o = oracle.build(pos, mass, n_leaf, lo=lo, side=side, curve=curve)
    g = gpu_build(pos, mass, n_leaf, box=((lo, side) if box == "given" else None), **kw)
    compare_structure(g, o)
    _, keys = oracle.keys(pos, lo, side, curve=curve)
    assert np.array_equal(g["key_sorted"], keys[o["perm"]])
    ext = cell_extents(pos, o, lo, side, curve) if extent else None
    em, ec, eq = moment_errors(g["com"], g["quad"], o["com"], o["quad"], o["cell_level"], side, ext)
    assert em <= FP64_TOL and ec <= FP64_TOL and eq <= FP64_TOL, (em, ec, eq)
    return g, o


# --------------------------------------------------------------------------
# small and ragged sizes
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 16, 17, 100, 1000, 2047, 2048, 2049, 4095, 4096, 4097,
                               10007, 65536, 100003])
def test_uniform_sizes(n):
    rng = _rng(n)
    pos = rng.random((n, 3), dtype=np.float32)
    mass = (rng.random(n) + 0.1).astype(np.float32)
    full_parity(pos, mass, 16)


@pytest.mark.parametrize("n_leaf", [1, 2, 8, 10, 16, 33, 64, 1024])
def test_n_leaf_values(n_leaf):
    pos, mass = dg.plummer(30000, seed=7)
    full_parity(pos, mass, n_leaf)


def test_config_uniform64k():
    pos, mass, nl = dg.workload("uniform64k")
    full_parity(pos, mass, nl)


def test_plummer_200k():
    pos, mass = dg.plummer(200000, seed=2)
    full_parity(pos, mass, 16)


def test_clustered_200k():
    pos, mass = dg.clustered(200000, seed=3, n_halos=200)
    full_parity(pos, mass, 8)


def test_exponential_disk():
    """The paper's second distribution: a thin disk (deep cells along z)."""
    pos, mass = dg.exponential_disk(200000, seed=6)
    full_parity(pos, mass, 16)
    full_parity(pos, mass, 10, subtrees=True)


def test_lognormal_masses():
    pos, mass = dg.clustered(100000, seed=5, n_halos=100, masses="lognormal")
    full_parity(pos, mass, 8)


# --------------------------------------------------------------------------
# degenerate cases
# --------------------------------------------------------------------------

def test_empty():
    g = gpu_build(np.zeros((0, 3), np.float32), np.zeros(0, np.float32), 16)
    assert g["n_cells"] == 0
    assert np.all(g["level_offset"] == 0)


def test_n_le_n_leaf_is_root_leaf():
    rng = _rng(3)
    for n in (1, 5, 16):
        g, o = full_parity(rng.random((n, 3), dtype=np.float32), np.ones(n, np.float32), 16)
        assert g["n_cells"] == 1 and g["child_ptr"][0, 0] == -1


def test_coincident_points_depth21_leaf():
    """More identical points than n_leaf: one saturated depth-21 leaf (the long
    leaf path), 22 cells in a chain."""
    pos = np.tile(np.array([[0.3, 0.7, 0.1]], np.float32), (5000, 1))
    mass = np.full(5000, 2.0 ** -12, np.float32)
    g, o = full_parity(pos, mass, 8)
    assert g["n_cells"] == 22 and g["cell_count"][21] == 5000


def test_duplicates_mixed():
    rng = _rng(12)
    base = rng.random((300, 3), dtype=np.float32)
    reps = rng.integers(1, 40, 300)
    pos = np.repeat(base, reps, axis=0)
    pos = pos[rng.permutation(pos.shape[0])]
    full_parity(pos, (rng.random(pos.shape[0]) + 0.5).astype(np.float32), 4)


def test_coincident_pairs_many_cells_per_tile():
    """Pairs of coincident points at n_leaf 1 each hang a chain of single-child
    cells down to depth 21.  Packed into one corner, they make the first tiles
    of 2048 sorted particles start several cells per particle (long per-thread
    runs of placements across many depths), while the uniform singles elsewhere
    start about one; both kinds of tile meet in one build."""
    rng = _rng(21)
    pairs = np.repeat((rng.random((3000, 3)) * 0.25).astype(np.float32), 2, axis=0)
    singles = rng.random((12000, 3), dtype=np.float32)
    pos = np.concatenate([pairs, singles])
    pos = pos[rng.permutation(pos.shape[0])]
    g, o = full_parity(pos, (rng.random(pos.shape[0]) + 0.5).astype(np.float32), 1)
    per_tile = np.bincount(o["cell_first"] // 2048)  # a cell starts at its first particle
    assert per_tile.max() > 8000 and per_tile.min() < 4000, per_tile


def test_complete_lattice():
    g1 = (np.arange(32) + 0.5) / 32
    pos = np.stack(np.meshgrid(g1, g1, g1, indexing="ij"), -1).reshape(-1, 3).astype(np.float32)
    g, o = full_parity(pos, np.ones(pos.shape[0], np.float32), 1)
    for d in range(6):
        assert g["level_offset"][d + 1] - g["level_offset"][d] == 8 ** d


def test_points_outside_box_clamp():
    """Out-of-box points are clamped into the edge cells for their keys; their
    moments use the true positions, so errors are measured against the extent
    of each cell's particles rather than the cell side."""
    rng = _rng(4)
    pos = (rng.random((20000, 3)) * 1.4 - 0.2).astype(np.float32)
    full_parity(pos, np.ones(20000, np.float32), 16, extent=True)


def test_nonunit_box():
    rng = _rng(5)
    pos = (rng.standard_normal((50000, 3)) * 10.0).astype(np.float32)
    pos = np.clip(pos, -60, 60)
    full_parity(pos, np.ones(50000, np.float32), 16, lo=(-64.0, -64.0, -64.0), side=128.0)


def test_auto_box():
    rng = _rng(6)
    pos = (rng.standard_normal((40000, 3)) * 3.0 + 7.0).astype(np.float32)
    lo, side = oracle.auto_box(pos)
    g, o = full_parity(pos, np.ones(40000, np.float32), 16, lo=lo, side=side, box="auto")
    assert np.array_equal(g["box"], np.array([*lo, side]))


# --------------------------------------------------------------------------
# mixed precision: FP32 + Kahan moments against the FP64 oracle
# --------------------------------------------------------------------------

MIXED_TOL = 1e-6


def mixed_parity(pos, mass, n_leaf, lo=(0.0, 0.0, 0.0), side=1.0):
    o = oracle.build(pos, mass, n_leaf, lo=lo, side=side)
    g = gpu_build(pos, mass, n_leaf, box=(lo, side), precision="mixed")
    compare_structure(g, o)  # the tree does not depend on the moment precision
    assert g["com"].dtype == np.float32 and g["quad"].dtype == np.float32
    em, ec, eq = moment_errors(g["com"].astype(np.float64), g["quad"].astype(np.float64),
                               o["com"], o["quad"], o["cell_level"], side)
    print(f"[mixed] N={pos.shape[0]} max rel err M={em:.2e} com={ec:.2e} Q={eq:.2e}", flush=True)
    assert em <= MIXED_TOL and ec <= MIXED_TOL and eq <= MIXED_TOL, (em, ec, eq)
    return em, ec, eq


def test_mixed_uniform64k():
    pos, mass, nl = dg.workload("uniform64k")
    mixed_parity(pos, mass, nl)


def test_mixed_plummer():
    pos, mass = dg.plummer(200000, seed=21)
    mixed_parity(pos, mass, 16)


def test_mixed_clustered_lognormal():
    pos, mass = dg.clustered(200000, seed=5, n_halos=200, masses="lognormal")
    mixed_parity(pos, mass, 8)


def test_mixed_nonunit_box_and_duplicates():
    rng = _rng(22)
    base = (rng.standard_normal((3000, 3)) * 5.0).astype(np.float32)
    pos = np.repeat(base, rng.integers(1, 12, 3000), axis=0)
    pos = np.clip(pos, -31, 31)
    mass = (rng.random(pos.shape[0]) + 0.01).astype(np.float32)
    mixed_parity(pos, mass, 4, lo=(-32.0, -32.0, -32.0), side=64.0)


# --------------------------------------------------------------------------
# determinism and options
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["default", "lookback", "counted"])
def test_perm_at_every_index_width(mode):
    """The radix passes pack key and index into one word once they fit, so the
    element formats change with the index width bits(N - 1).  N = 2^k and
    2^k + 1 for k = 0..20 runs every width up to 21 bits: perm must be the stable
    order of the oracle's keys, bit for bit, with the passes as the default
    picks them, with look-back and counted (TB_SORT_COUNTED)."""
    lookback, counted = mode == "lookback", mode == "counted"
    rng = np.random.default_rng(61)
    for k in range(0, 21):
        for n in sorted({1 << k, (1 << k) + 1}):
            pos = rng.random((n, 3), dtype=np.float32)
            pos[: n // 3] = pos[0]  # a third of the particles on one point: equal keys
            mass = np.full(n, 1.0 / n, np.float32)
            g = gpu_build(pos, mass, 16, lookback=lookback, counted=counted)
            _, keys = oracle.keys(pos)
            want = np.argsort(keys, kind="stable").astype(np.int32)
            assert np.array_equal(g["perm"], want), (n, mode)
            assert np.array_equal(g["key_sorted"], keys[want]), (n, mode)


def test_every_sort_config_identical():
    """Every sort shape, with its default passes (counted on small grids), with
    the look-back kept in every pass and with counting forced, gives the same
    tree."""
    pos, mass = dg.plummer(150000, seed=9)
    o = oracle.build(pos, mass, 16)
    ref = None
    for k in range(len(tb.tb_sort_configs())):
        for lookback, counted in ((False, False), (True, False), (False, True)):
            g = gpu_build(pos, mass, 16, sort_config=k, lookback=lookback, counted=counted)
            compare_structure(g, o)
            if ref is None:
                ref = g
            else:
                assert np.array_equal(g["com"], ref["com"]) and np.array_equal(g["quad"], ref["quad"])


def test_repeat_bit_identical():
    pos, mass = dg.plummer(120000, seed=10)
    p = torch.from_numpy(pos).cuda()
    m = torch.from_numpy(mass).cuda()
    b = tb.Builder(pos.shape[0], 16)
    outs = []
    for _ in range(3):
        b.launch(p, m, ((0, 0, 0), 1.0))
        r = b.result()
        outs.append({k: v.cpu().numpy() for k, v in r.items() if torch.is_tensor(v)})
    for k in outs[0]:
        for o in outs[1:]:
            assert np.array_equal(outs[0][k], o[k]), k


def test_sorted_particles_output():
    pos, mass = dg.plummer(50000, seed=11)
    p = torch.from_numpy(pos).cuda()
    m = torch.from_numpy(mass).cuda()
    r = tb.build(p, m, 16, ((0, 0, 0), 1.0), sorted_particles=True)
    perm = r["perm"].cpu().numpy()
    assert np.array_equal(r["pos_sorted"].cpu().numpy(), pos[perm])
    assert np.array_equal(r["mass_sorted"].cpu().numpy(), mass[perm])


def test_data_errors_reported():
    rng = _rng(13)
    pos = rng.random((5000, 3), dtype=np.float32)
    mass = np.ones(5000, np.float32)
    bad = pos.copy()
    bad[1234, 1] = np.nan
    with pytest.raises(tb.TreeBuildError) as e:
        gpu_build(bad, mass, 16)
    assert e.value.code == tb.TB_ERR_NONFINITE
    m2 = mass.copy()
    m2[77] = 0.0
    with pytest.raises(tb.TreeBuildError) as e:
        gpu_build(pos, m2, 16)
    assert e.value.code == tb.TB_ERR_MASS
    # a clean build on the same buffers afterwards clears the status word
    g = gpu_build(pos, mass, 16)
    assert g["n_cells"] > 1


# --------------------------------------------------------------------------
# full size: the benchmark configuration (N = 2^24 Plummer, n_leaf 16)
# --------------------------------------------------------------------------

@pytest.mark.timeout(1200)
def test_full_size_plummer_16m():
    """The headline configuration, every cell against a full oracle build: perm,
    keys and structure bit for bit, FP64 moments of all cells within 1e-12; for
    the default cell build and for the subtree-rooted one."""
    import time
    n = 1 << 24
    pos, mass, nl = dg.workload("plummer16m")
    print("[full] generated", flush=True)
    t0 = time.time()
    o = oracle.build(pos, mass, nl)
    print(f"[full] oracle built in {time.time() - t0:.1f} s, {o['n_cells']} cells", flush=True)
    _, keys = oracle.keys(pos)
    for subtrees in (False, True):
        g = gpu_build(pos, mass, nl, subtrees=subtrees)
        print(f"[full] built on the GPU (subtrees={subtrees}), {g['n_cells']} cells", flush=True)
        compare_structure(g, o)
        assert np.array_equal(g["key_sorted"], keys[o["perm"]])
        assert g["perm"].shape[0] == n
        em, ec, eq = moment_errors(g["com"], g["quad"], o["com"], o["quad"], o["cell_level"])
        print(f"[full] all {o['n_cells']} cells: max rel err M={em:.2e} com={ec:.2e} Q={eq:.2e}",
              flush=True)
        assert em <= FP64_TOL and ec <= FP64_TOL and eq <= FP64_TOL, (em, ec, eq)
        # the structural invariants, independently of the oracle
        tc.check_invariants(g, g["key_sorted"], nl)
        del g
