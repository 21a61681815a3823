"""Pins of the oracle's Peano-Hilbert keys (footnote of Sec. 2.2).

The curve is fixed by what makes it a Hilbert curve, checked exhaustively on
small grids: it visits every cell once, starts at the origin, and consecutive
cells share a face.  Its use as a hashed oct-tree key needs the prefix
property: the top 3d index bits of a point on the 21-level curve are the
index of its depth-d cell on the d-level curve, so a cell's key is a prefix of
its particles' keys as with Morton keys.  The tree built on Hilbert keys must
then be the Morton tree relabelled: the same geometric cells, each with the
same particles and moments, only listed in another order.
"""
import numpy as np
import pytest

import oracle
import treecheck as tc


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.mark.parametrize("bits", [1, 2, 3, 4])
def test_curve_visits_every_cell_once_by_face_steps(bits):
    n = 8 ** bits
    q = oracle.hilbert_decode(np.arange(n, dtype=np.uint64), bits).astype(np.int64)
    assert q.min() == 0 and q.max() == 2 ** bits - 1
    assert len({tuple(r) for r in q}) == n                      # a bijection
    assert np.array_equal(q[0], [0, 0, 0])                      # starts at the origin
    step = np.abs(np.diff(q, axis=0))
    assert np.all(step.sum(1) == 1) and np.all(step.max(1) == 1)  # face neighbours
    h = oracle.hilbert_encode(q.astype(np.uint32), bits)
    assert np.array_equal(h, np.arange(n, dtype=np.uint64))     # encode inverts decode


def test_curve_is_not_the_morton_order():
    """Two levels: Morton order jumps between non-adjacent cells; the curve never does."""
    q = oracle.hilbert_decode(np.arange(64, dtype=np.uint64), 2)
    morton = np.array([[(i >> 5 & 1) << 1 | (i >> 2 & 1), (i >> 4 & 1) << 1 | (i >> 1 & 1),
                        (i >> 3 & 1) << 1 | (i & 1)] for i in range(64)])
    assert not np.array_equal(q, morton)
    assert np.abs(np.diff(morton, axis=0)).sum(1).max() > 1


def test_round_trip_21_levels():
    q = _rng(1).integers(0, 2 ** 21, (20000, 3), dtype=np.uint32)
    h = oracle.hilbert_encode(q, 21)
    assert int(h.max()) < 2 ** 63
    assert np.array_equal(oracle.hilbert_decode(h, 21), q)


def test_prefix_is_the_coarse_curve_index():
    """The depth-d prefix of a 21-level index is the d-level index of the
    point's depth-d cell: a cell key is a prefix of its particles' keys."""
    rng = _rng(2)
    q = rng.integers(0, 2 ** 21, (5000, 3), dtype=np.uint32)
    h = oracle.hilbert_encode(q, 21)
    for d in range(0, 22):
        coarse = oracle.hilbert_encode(q >> np.uint32(21 - d), d)
        assert np.array_equal(h >> np.uint64(3 * (21 - d)), coarse), d


def test_keys_are_leading_one_plus_index():
    rng = _rng(3)
    pos = rng.random((3000, 3), dtype=np.float32)
    q, k = oracle.keys(pos, curve="hilbert")
    qm, _ = oracle.keys(pos)
    assert np.array_equal(q, qm)  # the same quantisation
    assert np.array_equal(k, np.uint64(1 << 63) | oracle.hilbert_encode(q, 21))


def _morton_ijk(key, d):
    ijk = [0, 0, 0]
    for l in range(d):
        digit = (key >> (3 * (d - 1 - l))) & 7
        for a in range(3):
            ijk[a] = (ijk[a] << 1) | ((digit >> (2 - a)) & 1)
    return ijk


def _geometric(t, curve):
    """(depth, i, j, k) of every cell of an oracle tree."""
    out = []
    for c in range(t["n_cells"]):
        key, d = int(t["cell_key"][c]), int(t["cell_level"][c])
        idx = key & ((1 << (3 * d)) - 1)
        if curve == "hilbert":
            ijk = tuple(int(v) for v in oracle.hilbert_decode(np.array([idx], np.uint64), d)[0])
        else:
            ijk = tuple(_morton_ijk(key, d))
        out.append((d, *ijk))
    return out


@pytest.mark.parametrize("seed,n,n_leaf", [(4, 400, 1), (5, 3000, 8), (6, 2000, 16)])
def test_hilbert_tree_is_the_morton_tree_relabelled(seed, n, n_leaf):
    rng = _rng(seed)
    pos = np.concatenate([rng.random((n // 2, 3)), 0.3 + 0.01 * rng.random((n - n // 2, 3))])
    pos = pos.astype(np.float32)
    mass = (rng.random(n) + 0.1).astype(np.float32)
    tm = oracle.build(pos, mass, n_leaf)
    th = oracle.build(pos, mass, n_leaf, curve="hilbert")
    assert th["n_cells"] == tm["n_cells"]
    assert np.array_equal(th["level_offset"], tm["level_offset"])
    gm = {g: c for c, g in enumerate(_geometric(tm, "morton"))}
    gh = _geometric(th, "hilbert")
    assert set(gh) == set(gm)
    for ch, g in enumerate(gh):
        cm = gm[g]
        fh, nh = int(th["cell_first"][ch]), int(th["cell_count"][ch])
        fm, nm = int(tm["cell_first"][cm]), int(tm["cell_count"][cm])
        assert nh == nm
        assert sorted(th["perm"][fh:fh + nh]) == sorted(tm["perm"][fm:fm + nm])
        assert (th["child_ptr"][ch, 1] == tm["child_ptr"][cm, 1])
        l = 2.0 ** -g[0]
        M = tm["com"][cm, 3]
        assert abs(th["com"][ch, 3] - M) <= 1e-14 * M
        assert np.abs(th["com"][ch, :3] - tm["com"][cm, :3]).max() <= 1e-14 * l
        assert np.abs(th["quad"][ch] - tm["quad"][cm]).max() <= 1e-13 * M * l * l
    # the structural invariants of a hashed oct-tree hold for the new keys
    _, keys = oracle.keys(pos, curve="hilbert")
    tc.check_invariants(th, keys[th["perm"]], n_leaf)


def test_hilbert_walk_equals_morton_walk():
    """The group walk visits the same cells in another order: the same forces."""
    rng = _rng(7)
    n = 3000
    pos = (0.5 + 0.15 * rng.standard_normal((n, 3))).clip(0.01, 0.99).astype(np.float32)
    mass = np.full(n, 1.0 / n, np.float32)
    tm = oracle.build(pos, mass, 8)
    th = oracle.build(pos, mass, 8, curve="hilbert")
    am, sm = oracle.walk_forces(pos, mass, tm, 0.6, 64, 1e-3)
    ah, sh = oracle.walk_forces(pos, mass, th, 0.6, 64, 1e-3, curve="hilbert")
    assert sm == sh
    om = np.empty_like(am)
    om[tm["perm"]] = am
    oh = np.empty_like(ah)
    oh[th["perm"]] = ah
    scale = np.abs(om[:, :3]).max()
    assert np.abs(om[:, :4] - oh[:, :4]).max() <= 1e-12 * scale
