"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* the paper's worked example of the minimum distinguished depth (Sec. 2.3.1);
* Morton keys derived by hand from the key definition (Sec. 2.2);
* the set-definition tree in exact rational geometry (Sec. 2.1);
* the leaf-first method written sequentially from Sec. 2.3.1-2.3.2 (Appendix A);
* closed forms: complete lattices, coincident points, tiny sets;
* moments in exact rational arithmetic, two-body and cubic-symmetric cases,
  power-of-two masses.
"""
import os

import numpy as np
import pytest

import oracle
import treecheck as tc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# keys
# --------------------------------------------------------------------------

def test_paper_min_depth_example():
    """Sec. 2.3.1: keys 1010011... and 1011011... separate at depth 1."""
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "paper_min_depth_example.txt"))
            if ln.strip() and not ln.startswith("#")]
    (a, b, md, ca, cb), = rows
    ka = int(a, 2) << (64 - len(a))
    kb = int(b, 2) << (64 - len(b))
    assert tc.min_depth(ka, kb) == int(md)
    assert tc.prefix_key(ka, 1) == int(ca, 2)
    assert tc.prefix_key(kb, 1) == int(cb, 2)
    assert tc.prefix_key(ka, 0) == tc.prefix_key(kb, 0) == 1
    # Points in those depth-1 octants (x lower, y upper, z lower / upper) give
    # oracle keys with those prefixes and, with n_leaf = 1, two depth-1 leaves.
    pos = np.array([[0.2, 0.6, 0.3], [0.2, 0.6, 0.7]], dtype=np.float32)
    _, k = oracle.keys(pos)
    assert int(k[0]) >> 60 == int(ca, 2) and int(k[1]) >> 60 == int(cb, 2)
    t = oracle.build(pos, np.ones(2, np.float32), n_leaf=1)
    assert t["n_cells"] == 3
    assert list(t["cell_level"]) == [0, 1, 1]
    assert [int(x) for x in t["cell_key"]] == [1, int(ca, 2), int(cb, 2)]


def test_hand_derived_keys():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "hand_keys.txt"))
            if ln.strip() and not ln.startswith("#")]
    pos = np.array([[float(r[0]), float(r[1]), float(r[2])] for r in rows], dtype=np.float32)
    want = np.array([int(r[3]) for r in rows], dtype=np.uint64)
    _, k = oracle.keys(pos)
    assert np.array_equal(k, want)


def test_keys_nonunit_box():
    """Scaling points and box by a power of two, or shifting both by an amount that
    keeps the FP32 coordinates exact, leaves the keys unchanged."""
    rng = _rng(3)
    p = (rng.integers(0, 2 ** 20, (500, 3)) * 2.0 ** -20).astype(np.float32)
    _, k0 = oracle.keys(p)
    _, k1 = oracle.keys(p * np.float32(4.0), side=4.0)
    assert np.array_equal(k0, k1)
    _, k2 = oracle.keys(p + np.float32(-8.0), lo=(-8, -8, -8), side=1.0)
    assert np.array_equal(k0, k2)


def test_key_prefix_is_geometric_cell():
    """The depth-d prefix of the oracle key equals the key of the depth-d cube
    that holds the point, built by appending octants (exact geometry)."""
    pos = _rng(5).random((40, 3), dtype=np.float32)
    _, k = oracle.keys(pos)
    g = tc.geometric_tree(pos, n_leaf=1)
    assert np.array_equal(k, g["particle_key"])


# --------------------------------------------------------------------------
# structure
# --------------------------------------------------------------------------

def _sets():
    rng = _rng(11)
    yield "uniform", rng.random((150, 3), dtype=np.float32), 4
    yield "tiny", rng.random((5, 3), dtype=np.float32), 1
    # clustered: power-law radii around a point, wide depth range
    r = rng.random(120) ** 6 * 0.4
    v = rng.standard_normal((120, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    yield "clustered", (0.5 + r[:, None] * v).astype(np.float32), 3
    # repeated points: more than n_leaf identical positions -> depth-21 leaves
    base = rng.random((6, 3), dtype=np.float32)
    rep = np.repeat(base, [1, 2, 7, 9, 1, 3], axis=0)
    yield "repeated", rep[rng.permutation(rep.shape[0])], 4
    # near-coincident points that split only at the deepest levels
    e = np.float32(2.0 ** -20)
    near = np.array([[0.3, 0.3, 0.3]] * 5, np.float32) + e * rng.integers(0, 3, (5, 3)).astype(np.float32)
    yield "near", np.concatenate([near, rng.random((10, 3), dtype=np.float32)]), 2
    yield "n_leaf_large", rng.random((30, 3), dtype=np.float32), 64


@pytest.mark.parametrize("name,pos,n_leaf", list(_sets()), ids=lambda v: v if isinstance(v, str) else "")
def test_oracle_equals_set_definition(name, pos, n_leaf):
    mass = np.ones(pos.shape[0], np.float32)
    t = oracle.build(pos, mass, n_leaf, moments=False)
    g = tc.geometric_tree(pos, n_leaf)
    assert t["n_cells"] == len(g["cells"])
    assert np.array_equal(t["perm"], g["perm"])
    assert np.array_equal(t["dfs_perm"], g["perm"])
    for c, cl in enumerate(g["cells"]):
        assert int(t["cell_key"][c]) == cl["key"]
        assert int(t["cell_level"][c]) == cl["level"]
        f, n = int(t["cell_first"][c]), int(t["cell_count"][c])
        assert n == len(cl["members"])
        assert list(t["perm"][f:f + n]) == cl["members"]
    _, keys = oracle.keys(pos)
    tc.check_invariants(t, keys[t["perm"]], n_leaf)


@pytest.mark.parametrize("seed", range(40))
def test_oracle_equals_paper_algorithms(seed):
    """Leaves and parents built the leaf-first way (Sec. 2.3.1-2.3.2, Algorithms
    1-2) equal the oracle's top-down tree."""
    rng = _rng(100 + seed)
    n = int(rng.integers(1, 200))
    n_leaf = int(rng.integers(1, 20))
    kind = seed % 4
    if kind == 0:
        pos = rng.random((n, 3), dtype=np.float32)
    elif kind == 1:
        r = rng.random(n) ** 8 * 0.5
        v = rng.standard_normal((n, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        pos = np.clip(0.5 + r[:, None] * v, 0, 0.999).astype(np.float32)
    elif kind == 2:
        base = rng.random((max(1, n // 10), 3), dtype=np.float32)
        pos = base[rng.integers(0, base.shape[0], n)]
    else:
        pos = (rng.integers(0, 8, (n, 3)) / 8.0 + 2.0 ** -22).astype(np.float32)
    mass = np.ones(n, np.float32)
    t = oracle.build(pos, mass, n_leaf, moments=False)
    _, keys = oracle.keys(pos)
    sk = keys[t["perm"]]
    leaves = tc.leaves_from_sorted_keys(sk, n_leaf)
    cells = tc.parents_bottom_up(leaves)
    assert len(cells) == t["n_cells"]
    for c in range(t["n_cells"]):
        d, k = int(t["cell_level"][c]), int(t["cell_key"][c])
        cl = cells[(d, k)]
        assert cl["first"] == t["cell_first"][c]
        assert cl["count"] == t["cell_count"][c]
        assert cl["leaf"] == (t["child_ptr"][c, 0] < 0)
        if not cl["leaf"]:
            f, m = t["child_ptr"][c]
            assert [int(x) for x in t["cell_key"][f:f + m]] == cl["children"]


def test_insertion_order_invariance():
    rng = _rng(21)
    pos = rng.random((300, 3), dtype=np.float32)
    mass = rng.random(300).astype(np.float32) + 0.5
    t0 = oracle.build(pos, mass, 5)
    p = rng.permutation(300)
    t1 = oracle.build(pos[p], mass[p], 5)
    for k in ("cell_key", "cell_level", "cell_first", "cell_count", "child_ptr"):
        assert np.array_equal(t0[k], t1[k])
    # same particles in the same sorted slots (no duplicate keys here)
    assert np.array_equal(p[t1["perm"]], t0["perm"])
    np.testing.assert_allclose(t0["com"], t1["com"], rtol=0, atol=1e-15)


def test_complete_lattice_closed_form():
    """2^k points per axis at cell centres with n_leaf = 1: a complete oct-tree with
    8^d cells at depth d for d <= k."""
    for k in (1, 2, 3):
        g = (np.arange(2 ** k) + 0.5) / 2 ** k
        pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.float32)
        t = oracle.build(pos, np.ones(pos.shape[0], np.float32), 1, moments=False)
        loff = t["level_offset"]
        for d in range(k + 1):
            assert loff[d + 1] - loff[d] == 8 ** d
        assert t["n_cells"] == sum(8 ** d for d in range(k + 1))
        assert np.all(t["cell_count"][loff[k]:loff[k + 1]] == 1)


def test_coincident_points_closed_form():
    """n > n_leaf identical points: a chain of single-child cells down to one
    depth-21 leaf holding all of them."""
    pos = np.tile(np.array([[0.3, 0.7, 0.1]], np.float32), (40, 1))
    t = oracle.build(pos, np.ones(40, np.float32), 8)
    assert t["n_cells"] == 22
    assert list(t["cell_level"]) == list(range(22))
    assert np.all(t["cell_count"] == 40)
    assert np.array_equal(t["perm"], np.arange(40))
    assert t["child_ptr"][21, 0] == -1
    assert np.all(t["child_ptr"][:21, 1] == 1)


def test_small_sets():
    t = oracle.build(np.zeros((0, 3), np.float32), np.zeros(0, np.float32), 4)
    assert t["n_cells"] == 0
    pos = _rng(1).random((4, 3), dtype=np.float32)
    t = oracle.build(pos, np.ones(4, np.float32), 4)
    assert t["n_cells"] == 1 and t["cell_count"][0] == 4 and t["child_ptr"][0, 0] == -1
    t = oracle.build(pos[:1], np.ones(1, np.float32), 1)
    assert t["n_cells"] == 1


def test_max_cells_bound():
    for n, nl in [(1, 1), (100, 1), (1000, 16), (12345, 8)]:
        assert oracle.max_cells(n, nl) == n + 21 * (n // (nl + 1))
    rng = _rng(7)
    pos = np.repeat(rng.random((30, 3), dtype=np.float32), 2, axis=0)
    t = oracle.build(pos, np.ones(60, np.float32), 1, moments=False)
    assert t["n_cells"] <= oracle.max_cells(60, 1)


def test_error_codes():
    pos = np.zeros((3, 3), np.float32)
    with pytest.raises(oracle.OracleError) as e:
        oracle.build(pos, np.ones(3, np.float32), 4, side=3.0)
    assert e.value.code == -2
    bad = pos.copy()
    bad[1, 2] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.build(bad, np.ones(3, np.float32), 4)
    assert e.value.code == -5
    with pytest.raises(oracle.OracleError) as e:
        oracle.build(pos, np.array([1, 0, 1], np.float32), 4)
    assert e.value.code == -6
    with pytest.raises(oracle.OracleError):
        oracle.build(pos, np.ones(3, np.float32), 0)


def test_auto_box():
    pos = np.array([[0.1, 0.2, 0.3], [0.6, 0.2, 0.35]], np.float32)
    lo, side = oracle.auto_box(pos)
    assert np.array_equal(lo, pos.min(0).astype(np.float64)) and side == 1.0
    lo, side = oracle.auto_box(pos * np.float32(100))
    assert side == 64.0
    lo, side = oracle.auto_box(pos[:1])
    assert side == 1.0
    lo, side = oracle.auto_box(np.array([[0, 0, 0], [0.5, 0, 0]], np.float32))
    assert side == 1.0  # smallest power of two strictly above 0.5


# --------------------------------------------------------------------------
# moments
# --------------------------------------------------------------------------

def _rel_errors(com, quad, M, c_ex, q_ex, level, side=1.0):
    l = side / 2 ** level
    e_m = abs(com[3] - float(M)) / float(M)
    e_c = max(abs(com[a] - float(c_ex[a])) for a in range(3)) / l
    e_q = max(abs(quad[i] - float(q_ex[i])) for i in range(6)) / (float(M) * l * l)
    return e_m, e_c, e_q


@pytest.mark.parametrize("seed", range(6))
def test_moments_exact_rationals(seed):
    rng = _rng(200 + seed)
    n = 60
    if seed % 2:
        pos = rng.random((n, 3), dtype=np.float32)
    else:
        pos = (0.3 + 1e-3 * rng.random((n, 3))).astype(np.float32)
    mass = (rng.random(n) + 0.1).astype(np.float32)
    t = oracle.build(pos, mass, 3)
    for c in range(t["n_cells"]):
        f, cnt = int(t["cell_first"][c]), int(t["cell_count"][c])
        mem = list(t["perm"][f:f + cnt])
        M, cx, qx = tc.exact_moments(pos, mass, mem, int(t["cell_key"][c]), int(t["cell_level"][c]))
        em, ec, eq = _rel_errors(t["com"][c], t["quad"][c], M, cx, qx, int(t["cell_level"][c]))
        assert em < 1e-15 and ec < 1e-15 and eq < 1e-14, (c, em, ec, eq)


def test_moments_nonunit_box_exact():
    rng = _rng(9)
    pos = (rng.random((40, 3)) * 3.0 - 1.5).astype(np.float32)
    mass = (rng.random(40) + 0.1).astype(np.float32)
    lo = (-2.0, -2.0, -2.0)
    t = oracle.build(pos, mass, 2, lo=lo, side=4.0)
    for c in range(t["n_cells"]):
        f, cnt = int(t["cell_first"][c]), int(t["cell_count"][c])
        M, cx, qx = tc.exact_moments(pos, mass, list(t["perm"][f:f + cnt]), int(t["cell_key"][c]),
                                     int(t["cell_level"][c]), lo=lo, side=4.0)
        em, ec, eq = _rel_errors(t["com"][c], t["quad"][c], M, cx, qx, int(t["cell_level"][c]), 4.0)
        assert em < 1e-15 and ec < 1e-15 and eq < 1e-14


def test_two_body_quadrupole():
    """Two bodies: Q = mu (3 s s - s^2 delta) with mu = m1 m2 / (m1 + m2)."""
    p = np.array([[0.1, 0.2, 0.3], [0.35, 0.15, 0.4]], np.float32)
    m = np.array([0.25, 0.75], np.float32)
    t = oracle.build(p, m, 2)
    s = p[0].astype(np.float64) - p[1].astype(np.float64)
    mu = 0.25 * 0.75 / 1.0
    s2 = s @ s
    want = mu * np.array([3 * s[0] * s[0] - s2, 3 * s[0] * s[1], 3 * s[0] * s[2],
                          3 * s[1] * s[1] - s2, 3 * s[1] * s[2], 3 * s[2] * s[2] - s2])
    np.testing.assert_allclose(t["quad"][0], want, rtol=1e-14, atol=1e-17)
    com_abs = (0.25 * p[0].astype(np.float64) + 0.75 * p[1].astype(np.float64))
    np.testing.assert_allclose(t["com"][0, :3], com_abs - 0.5, rtol=0, atol=1e-16)
    assert t["com"][0, 3] == 1.0


def test_cubic_symmetric_cell():
    """8 equal masses at the corners of a cube centred on a cell centre: com at the
    centre, traceless quadrupole zero."""
    d = 0.125
    c = np.array([0.25, 0.75, 0.25])
    pos = np.array([c + d * np.array(s) for s in np.ndindex(2, 2, 2)], np.float64)
    pos = (pos - d / 2).astype(np.float32)
    pos = np.array([c + d * (2 * np.array(s) - 1) / 2 for s in np.ndindex(2, 2, 2)]).astype(np.float32)
    t = oracle.build(pos, np.full(8, 0.125, np.float32), 8)
    # root cell holds all 8 (n_leaf = 8): centre of the root is 0.5
    np.testing.assert_array_equal(t["com"][0, :3], c - 0.5)
    assert np.all(t["quad"][0] == 0.0)


def test_power_of_two_masses_exact():
    rng = _rng(4)
    pos = rng.random((257, 3), dtype=np.float32)
    m = np.full(257, 2.0 ** -9, np.float32)
    t = oracle.build(pos, m, 4)
    assert np.array_equal(t["com"][:, 3], t["cell_count"] * 2.0 ** -9)
    # single-particle leaves: com_rel = position minus centre exactly, Q = 0 exactly
    one = np.nonzero((t["cell_count"] == 1))[0]
    assert one.size > 0
    for c in one[:50]:
        p = t["perm"][t["cell_first"][c]]
        off = np.array([float(v) for v in tc.cell_centre_offset(int(t["cell_key"][c]),
                                                                int(t["cell_level"][c]), 1.0)])
        assert np.array_equal(t["com"][c, :3], pos[p].astype(np.float64) - off)
        assert np.all(t["quad"][c] == 0.0)


def test_root_matches_global_sums():
    rng = _rng(8)
    pos = rng.random((2000, 3), dtype=np.float32)
    mass = (rng.random(2000) + 0.01).astype(np.float32)
    t = oracle.build(pos, mass, 16)
    import math
    M = math.fsum(mass.astype(np.float64))
    assert abs(t["com"][0, 3] - M) <= 1e-15 * M
    for a in range(3):
        ca = math.fsum(mass.astype(np.float64) * pos[:, a].astype(np.float64)) / M - 0.5
        assert abs(t["com"][0, a] - ca) < 1e-15
    assert abs(t["quad"][0, 0] + t["quad"][0, 3] + t["quad"][0, 5]) < 1e-15 * M


# --------------------------------------------------------------------------
# the single-cell moment wrapper (used by the large sampled parity checks)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_cell_moments_every_cell(seed):
    """oracle.cell_moments, given each cell's own range of the oracle's perm and
    the cell's key and depth, returns the build's moments bit for bit, and both
    equal the exact rational moments of the cell's particles.  Odd seeds use a
    non-unit box, so a dropped box corner or side also fails."""
    rng = _rng(300 + seed)
    n = 70
    if seed % 2:
        lo, side = (-4.0, -4.0, -4.0), 8.0
        pos = (rng.random((n, 3)) * 6.0 - 3.0).astype(np.float32)
    else:
        lo, side = (0.0, 0.0, 0.0), 1.0
        pos = rng.random((n, 3), dtype=np.float32)
    mass = (rng.random(n) + 0.1).astype(np.float32)
    t = oracle.build(pos, mass, 2, lo=lo, side=side)
    for c in range(t["n_cells"]):
        f, cnt = int(t["cell_first"][c]), int(t["cell_count"][c])
        key, lvl = int(t["cell_key"][c]), int(t["cell_level"][c])
        com, quad = oracle.cell_moments(pos, mass, t["perm"], f, cnt, key, lvl, lo=lo, side=side)
        assert np.array_equal(com, t["com"][c]) and np.array_equal(quad, t["quad"][c]), c
        M, cx, qx = tc.exact_moments(pos, mass, list(t["perm"][f:f + cnt]), key, lvl, lo=lo,
                                     side=side)
        em, ec, eq = _rel_errors(com, quad, M, cx, qx, lvl, side)
        assert em < 1e-15 and ec < 1e-15 and eq < 1e-14, (c, em, ec, eq)


def test_cell_moments_argument_roles():
    """A range that is not the cell's, or the right range in another cell's frame,
    gives other moments: first/count, key and depth each matter."""
    rng = _rng(310)
    pos = rng.random((200, 3), dtype=np.float32)
    mass = (rng.random(200) + 0.1).astype(np.float32)
    t = oracle.build(pos, mass, 4)
    c = int(np.nonzero((t["cell_level"] == 2) & (t["cell_count"] > 3))[0][0])
    f, cnt = int(t["cell_first"][c]), int(t["cell_count"][c])
    key, lvl = int(t["cell_key"][c]), int(t["cell_level"][c])
    ref_c, ref_q = oracle.cell_moments(pos, mass, t["perm"], f, cnt, key, lvl)
    M, cx, _ = tc.exact_moments(pos, mass, list(t["perm"][f:f + cnt]), key, lvl)
    assert abs(ref_c[3] - float(M)) <= 1e-15 * float(M)
    for args in [(f + 1, cnt - 1, key, lvl), (f, cnt, key ^ 1, lvl), (f, cnt, key >> 3, lvl - 1)]:
        oc, oq = oracle.cell_moments(pos, mass, t["perm"], *args)
        assert not (np.array_equal(oc, ref_c) and np.array_equal(oq, ref_q)), args


# --------------------------------------------------------------------------
# the paper's own method on one CPU thread (second CPU reference)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(24))
def test_leaf_first_reference_equals_oracle(seed):
    """The sequential leaf-first build (Sec. 2.3, Algorithms 1 and 2, moments
    combined from the children) gives the oracle's tree bit for bit and its
    moments to rounding, on adversarial tiny inputs."""
    rng = _rng(400 + seed)
    n = int(rng.integers(1, 300))
    n_leaf = int(rng.integers(1, 20))
    kind = seed % 4
    if kind == 0:
        pos = rng.random((n, 3), dtype=np.float32)
    elif kind == 1:
        r = rng.random(n) ** 8 * 0.5
        v = rng.standard_normal((n, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        pos = np.clip(0.5 + r[:, None] * v, 0, 0.999).astype(np.float32)
    elif kind == 2:
        base = rng.random((max(1, n // 10), 3), dtype=np.float32)
        pos = base[rng.integers(0, base.shape[0], n)]
    else:
        pos = (rng.integers(0, 8, (n, 3)) / 8.0 + 2.0 ** -22).astype(np.float32)
    mass = (rng.random(n) + 0.05).astype(np.float32)
    a = oracle.build(pos, mass, n_leaf)
    b = oracle.leaf_first_build(pos, mass, n_leaf)
    for k in ("perm", "cell_key", "cell_level", "cell_first", "cell_count", "child_ptr",
              "level_offset"):
        assert np.array_equal(a[k], b[k]), k
    lvl = a["cell_level"].astype(np.int64)
    l = np.ldexp(1.0, -lvl)
    M = a["com"][:, 3]
    assert np.max(np.abs(b["com"][:, 3] - M) / M) <= 1e-14
    assert np.max(np.abs(b["com"][:, :3] - a["com"][:, :3]).max(1) / l) <= 1e-14
    assert np.max(np.abs(b["quad"] - a["quad"]).max(1) / (M * l * l)) <= 1e-13


def test_leaf_first_reference_degenerate():
    """Empty set, a root leaf, and coincident points (a saturated depth-21 leaf)."""
    e = oracle.leaf_first_build(np.zeros((0, 3), np.float32), np.zeros(0, np.float32), 4)
    assert e["n_cells"] == 0
    pos = _rng(5).random((3, 3), dtype=np.float32)
    r = oracle.leaf_first_build(pos, np.ones(3, np.float32), 4)
    assert r["n_cells"] == 1 and r["child_ptr"][0, 0] == -1 and r["cell_key"][0] == 1
    pos = np.tile(np.array([[0.3, 0.7, 0.1]], np.float32), (40, 1))
    r = oracle.leaf_first_build(pos, np.full(40, 0.25, np.float32), 8)
    assert r["n_cells"] == 22 and np.all(r["cell_count"] == 40)
    assert np.all(r["quad"] == 0.0) and np.all(r["com"][:, 3] == 10.0)


# --------------------------------------------------------------------------
# subtree-rooted build (Sec. 2.3.3, eq. 2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(30))
def test_subtree_rooted_build_equals_oracle(seed):
    """Blocks of at most n_serial particles, each built alone with the leaf depth
    of eq. 2 (d_root), plus the cells above the block roots, give exactly the
    oracle's tree; every block is one of its cells."""
    rng = _rng(500 + seed)
    n = int(rng.integers(1, 400))
    n_leaf = int(rng.integers(1, 12))
    n_serial = int(rng.integers(n_leaf, 4 * n_leaf + 30))
    kind = seed % 4
    if kind == 0:
        pos = rng.random((n, 3), dtype=np.float32)
    elif kind == 1:
        r = rng.random(n) ** 8 * 0.5
        v = rng.standard_normal((n, 3))
        v /= np.linalg.norm(v, axis=1)[:, None]
        pos = np.clip(0.5 + r[:, None] * v, 0, 0.999).astype(np.float32)
    elif kind == 2:
        base = rng.random((max(1, n // 12), 3), dtype=np.float32)
        pos = base[rng.integers(0, base.shape[0], n)]
    else:
        pos = (rng.integers(0, 8, (n, 3)) / 8.0 + 2.0 ** -22).astype(np.float32)
    t = oracle.build(pos, np.ones(n, np.float32), n_leaf, moments=False)
    _, keys = oracle.keys(pos)
    sk = keys[t["perm"]]
    cells = tc.subtree_build(sk, n_leaf, n_serial)
    assert len(cells) == t["n_cells"]
    index = {(int(t["cell_level"][c]), int(t["cell_key"][c])): c for c in range(t["n_cells"])}
    for (d, k), cl in cells.items():
        c = index[(d, k)]
        assert cl["first"] == t["cell_first"][c] and cl["count"] == t["cell_count"][c]
        assert cl["leaf"] == (t["child_ptr"][c, 0] < 0)
        if not cl["leaf"]:
            f, m = t["child_ptr"][c]
            assert [int(x) for x in t["cell_key"][f:f + m]] == cl["children"]
    for s, e, d_root in tc.subtree_blocks(sk, n_serial):
        c = index[(d_root, tc.prefix_key(int(sk[s]), d_root))]
        assert t["cell_first"][c] == s and t["cell_count"][c] == e - s
        assert e - s <= n_serial or d_root == 21


def test_eq2_needs_d_root():
    """Without the d_root term, a block of at most n_leaf particles read on its own
    has neither neighbour term (its first particle has no left neighbour inside
    the block and no particle n_leaf places further), so it would become a leaf
    at depth 0 instead of the leaf at the block root."""
    rng = _rng(77)
    pos = rng.random((300, 3), dtype=np.float32)
    t = oracle.build(pos, np.ones(300, np.float32), 4, moments=False)
    _, keys = oracle.keys(pos)
    sk = keys[t["perm"]]
    blocks = tc.subtree_blocks(sk, 20)
    s, e, d_root = next(b for b in blocks if b[2] > 0 and b[1] - b[0] <= 4)
    with_root = tc.leaves_in_block(sk[s:e], 4, d_root)
    without = tc.leaves_in_block(sk[s:e], 4, 0)
    assert with_root == [(d_root, tc.prefix_key(int(sk[s]), d_root), 0, e - s)]
    assert without == [(0, 1, 0, e - s)]
