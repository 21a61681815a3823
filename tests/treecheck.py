"""Independent checks used to pin the oracle (and, for invariants, the HIP path).

Nothing here imports the oracle or the product package.  Each routine derives
its result a different way from the oracle's top-down insertion:

* ``geometric_tree``  -- the set definition of the Barnes-Hut tree (Sec. 2.1),
  evaluated with exact rational geometry: a depth-d cell is the cube
  [i, i+1) x [j, j+1) x [k, k+1) scaled by side/2^d, it exists when its parent
  holds more than n_leaf particles, and its key is built by appending the
  3-bit octant to the parent key (Sec. 2.2).
* ``leaves_from_sorted_keys`` / ``parents_bottom_up`` -- the leaf-first method
  as the text of Sec. 2.3.1 and 2.3.2 describes it, written sequentially:
  leaves one after another from sorted keys with the leaf-depth formula proved
  in Appendix A, then parents one depth at a time from runs of equal key >> 3.
* ``exact_moments`` -- monopole, centre of mass and traceless quadrupole of a
  particle set in exact rational arithmetic (fractions.Fraction).
* ``check_invariants`` -- structural properties every correct tree has.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

MAX_DEPTH = 21


# ---------------------------------------------------------------------------
# geometric (set-definition) tree
# ---------------------------------------------------------------------------

def _cell_index(x: Fraction, lo: Fraction, side: Fraction, depth: int) -> int:
    """floor((x - lo) * 2^depth / side), clamped into [0, 2^depth - 1] (exact)."""
    t = (x - lo) * (1 << depth) / side
    i = t.numerator // t.denominator
    return min(max(i, 0), (1 << depth) - 1)


def geometric_tree(pos, n_leaf: int, lo=(0.0, 0.0, 0.0), side: float = 1.0):
    """Tree by the set definition, cells in (depth, key) order.

    Returns dict(cells=list of dict(level, key, members (sorted by particle key
    then index)), perm, particle_key)."""
    pos = np.asarray(pos, dtype=np.float32).reshape(-1, 3)
    n = pos.shape[0]
    flo = [Fraction(float(v)) for v in lo]
    fside = Fraction(float(side))
    fx = [[Fraction(float(pos[p, a])) for a in range(3)] for p in range(n)]

    def ijk(p, d):
        return tuple(_cell_index(fx[p][a], flo[a], fside, d) for a in range(3))

    def child_key(parent_key, c):
        # the octant's 3-bit digit: x half, y half, z half (upper half = 1)
        return (parent_key << 3) | ((c[0] & 1) << 2) | ((c[1] & 1) << 1) | (c[2] & 1)

    # particle keys: depth-21 cell key, built one level at a time
    pkey = []
    for p in range(n):
        k = 1
        for d in range(1, MAX_DEPTH + 1):
            k = child_key(k, ijk(p, d))
        pkey.append(k)

    cells = []
    if n == 0:
        return dict(cells=cells, perm=np.zeros(0, np.int32), particle_key=np.zeros(0, np.uint64))

    frontier = [(0, 1, (0, 0, 0), list(range(n)))]
    while frontier:
        nxt = []
        for level, key, c, members in frontier:
            cells.append(dict(level=level, key=key, members=members))
            if len(members) > n_leaf and level < MAX_DEPTH:
                groups = {}
                for p in members:
                    groups.setdefault(ijk(p, level + 1), []).append(p)
                for cc, mem in groups.items():
                    nxt.append((level + 1, child_key(key, cc), cc, mem))
        frontier = nxt
    cells.sort(key=lambda cl: (cl["level"], cl["key"]))
    for cl in cells:
        cl["members"] = sorted(cl["members"], key=lambda p: (pkey[p], p))
    perm = sorted(range(n), key=lambda p: (pkey[p], p))
    return dict(cells=cells, perm=np.asarray(perm, np.int32),
                particle_key=np.asarray(pkey, dtype=np.uint64))


# ---------------------------------------------------------------------------
# the leaf-first method, sequentially (Sec. 2.3.1-2.3.2)
# ---------------------------------------------------------------------------

def clz64(x: int) -> int:
    return 64 - int(x).bit_length()


def min_depth(ki: int, kj: int) -> int:
    """Minimum distinguished depth: leading zero bits of the XOR, divided by three
    and rounded up (clz of 0 taken as 64)."""
    z = clz64(int(ki) ^ int(kj))
    return -(-z // 3)


def prefix_key(key: int, d: int) -> int:
    """Key of the depth-d cell holding a particle: the upper 3d+1 bits (Sec. 2.3.1)."""
    return int(key) >> (64 - (3 * d + 1))


def leaves_from_sorted_keys(sorted_keys, n_leaf: int):
    """Leaves read off sorted keys as Sec. 2.3.1 describes them, one leaf after
    another: the first particle of a leaf fixes the leaf depth as the larger of
    its minimum distinguished depth to the previous particle and to the particle
    n_leaf places further on (either missing at the ends counts as 0; depth
    capped at the 21-bit key resolution), and the leaf takes every following
    particle whose key has the same prefix at that depth.
    Returns [(depth, key, first, count)] in key order."""
    keys = [int(x) for x in sorted_keys]
    n = len(keys)
    out = []
    start = 0
    while start < n:
        left = min_depth(keys[start - 1], keys[start]) if start > 0 else 0
        right = min_depth(keys[start], keys[start + n_leaf]) if start + n_leaf < n else 0
        depth = min(max(left, right), MAX_DEPTH)
        prefix = prefix_key(keys[start], depth)
        stop = start + 1
        while stop < n and prefix_key(keys[stop], depth) == prefix:
            stop += 1
        out.append((depth, prefix, start, stop - start))
        start = stop
    return out


def parents_bottom_up(leaves):
    """All cells from the leaves, one depth at a time from the deepest, as
    Sec. 2.3.2 describes it: the cells of a depth (its leaves and the parents
    made one step earlier) in key order fall into runs sharing key >> 3; every
    run becomes one parent one depth up, with the run as its children.
    Returns {(depth, key): dict(first, count, children=[keys], leaf)}."""
    cells = {}
    at_depth = {}
    for d, key, first, count in leaves:
        cells[(d, key)] = dict(first=first, count=count, children=[], leaf=True)
        at_depth.setdefault(d, []).append(key)
    deepest = max((d for d, *_ in leaves), default=0)
    for d in range(deepest, 0, -1):
        run_key, run = None, []
        for key in sorted(at_depth.get(d, [])) + [None]:
            up = None if key is None else key >> 3
            if run and up != run_key:
                kids = [cells[(d, k)] for k in run]
                cells[(d - 1, run_key)] = dict(first=min(c["first"] for c in kids),
                                               count=sum(c["count"] for c in kids),
                                               children=list(run), leaf=False)
                at_depth.setdefault(d - 1, []).append(run_key)
                run = []
            run_key = up
            if key is not None:
                run.append(key)
    return cells


# ---------------------------------------------------------------------------
# exact moments
# ---------------------------------------------------------------------------

def cell_centre_offset(key: int, level: int, side: float):
    """Geometric centre of a cell relative to the box corner, from its key."""
    ijk = [0, 0, 0]
    for l in range(level):
        digit = (int(key) >> (3 * (level - 1 - l))) & 7
        ijk[0] = (ijk[0] << 1) | ((digit >> 2) & 1)
        ijk[1] = (ijk[1] << 1) | ((digit >> 1) & 1)
        ijk[2] = (ijk[2] << 1) | (digit & 1)
    h = Fraction(float(side)) / (1 << level)
    return [(Fraction(v) + Fraction(1, 2)) * h for v in ijk]


def exact_moments(pos, mass, members, key: int, level: int, lo=(0.0, 0.0, 0.0), side=1.0):
    """(M, com_rel[3], Q[6]) of the given particles in exact rationals.  com_rel is
    relative to the cell centre; Q = sum m (3 r_a r_b - r^2 delta_ab) about com."""
    off = cell_centre_offset(key, level, side)
    flo = [Fraction(float(v)) for v in lo]
    M = Fraction(0)
    s1 = [Fraction(0)] * 3
    rel = []
    for p in members:
        m = Fraction(float(mass[p]))
        r = [Fraction(float(pos[p][a])) - flo[a] - off[a] for a in range(3)]
        rel.append((m, r))
        M += m
        s1 = [s1[a] + m * r[a] for a in range(3)]
    com = [s / M for s in s1]
    q = [Fraction(0)] * 6
    for m, r in rel:
        d = [r[a] - com[a] for a in range(3)]
        d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
        q[0] += m * (3 * d[0] * d[0] - d2)
        q[1] += m * (3 * d[0] * d[1])
        q[2] += m * (3 * d[0] * d[2])
        q[3] += m * (3 * d[1] * d[1] - d2)
        q[4] += m * (3 * d[1] * d[2])
        q[5] += m * (3 * d[2] * d[2] - d2)
    return M, com, q


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------

def check_invariants(tree: dict, sorted_keys: np.ndarray, n_leaf: int):
    """Assert the structural properties of a (depth, key)-ordered tree.

    tree: cell_key, cell_level, cell_first, cell_count, child_ptr [C,2],
    level_offset [23], n_cells.  sorted_keys: particle keys in perm order."""
    key = np.asarray(tree["cell_key"], dtype=np.uint64)
    lvl = np.asarray(tree["cell_level"]).astype(np.int64)
    first = np.asarray(tree["cell_first"]).astype(np.int64)
    cnt = np.asarray(tree["cell_count"]).astype(np.int64)
    child = np.asarray(tree["child_ptr"]).astype(np.int64).reshape(-1, 2)
    loff = np.asarray(tree["level_offset"]).astype(np.int64)
    C = int(tree["n_cells"])
    n = len(sorted_keys)
    sk = np.asarray(sorted_keys, dtype=np.uint64)
    assert key.shape[0] == C
    if n == 0:
        assert C == 0
        return
    assert np.all(sk[1:] >= sk[:-1])
    # root
    assert lvl[0] == 0 and int(key[0]) == 1 and first[0] == 0 and cnt[0] == n
    # (depth, key) order and level offsets
    assert np.all(np.diff(lvl) >= 0)
    for d in range(22):
        a, b = loff[d], loff[d + 1]
        assert a <= b
        assert np.all(lvl[a:b] == d)
        if b - a > 1:
            assert np.all(key[a + 1:b] > key[a:b - 1])
    assert loff[22] == C
    # every cell key is the depth prefix of its particles' keys
    shift = (63 - 3 * lvl).astype(np.uint64)
    assert np.all((sk[first] >> shift) == key)
    last = first + cnt - 1
    assert np.all((sk[last] >> shift) == key)
    # ranges are maximal: neighbours outside the range have another prefix
    before = first > 0
    assert np.all((sk[first[before] - 1] >> shift[before]) != key[before])
    after = last < n - 1
    assert np.all((sk[last[after] + 1] >> shift[after]) != key[after])
    # leaves partition the particles; internal cells hold more than n_leaf
    is_leaf = child[:, 0] < 0
    assert np.all(child[is_leaf, 1] == 0)
    order = np.argsort(first[is_leaf], kind="stable")
    lf, lc = first[is_leaf][order], cnt[is_leaf][order]
    assert lf[0] == 0 and np.all(lf[1:] == lf[:-1] + lc[:-1]) and lf[-1] + lc[-1] == n
    assert np.all((cnt[is_leaf] <= n_leaf) | (lvl[is_leaf] == MAX_DEPTH))
    assert np.all(cnt[~is_leaf] > n_leaf) and np.all(lvl[~is_leaf] < MAX_DEPTH)
    # children partition their parent, keys extend the parent key
    inner = np.nonzero(~is_leaf)[0]
    if inner.size == 0:
        assert C == 1
        return
    nch = child[inner, 1]
    assert np.all((nch >= 1) & (nch <= 8))
    fc = child[inner, 0]
    assert np.all(lvl[fc] == lvl[inner] + 1)
    par = np.repeat(inner, nch)
    ch = np.repeat(fc - np.concatenate([[0], np.cumsum(nch)[:-1]]), nch) + np.arange(nch.sum())
    assert np.all((key[ch] >> np.uint64(3)) == key[par])
    is_first = np.zeros(ch.shape[0], dtype=bool)
    is_first[np.concatenate([[0], np.cumsum(nch)[:-1]])] = True
    assert np.all(first[ch[is_first]] == first[inner])
    nf = ~is_first
    assert np.all(first[ch[nf]] == first[ch[nf] - 1] + cnt[ch[nf] - 1])
    sums = np.zeros(C, dtype=np.int64)
    np.add.at(sums, par, cnt[ch])
    assert np.all(sums[inner] == cnt[inner])
    # every non-root cell is somebody's child exactly once
    parent_count = np.zeros(C, dtype=np.int64)
    np.add.at(parent_count, ch, 1)
    assert parent_count[0] == 0 and np.all(parent_count[1:] == 1)


# ---------------------------------------------------------------------------
# subtree-rooted build (Sec. 2.3.3, eq. 2), sequentially
# ---------------------------------------------------------------------------

def subtree_blocks(sorted_keys, n_serial: int):
    """Sec. 2.3.3: divide the sorted keys recursively into blocks until each block
    is a subtree of at most n_serial particles, splitting a range by the next
    3-bit digit of its keys (so no two blocks share a cell).  A range of
    identical keys at depth 21 cannot be divided and stays one block.
    Returns [(first, end, d_root)] in key order."""
    keys = [int(x) for x in sorted_keys]
    out = []

    def divide(s, e, d):
        if e - s <= n_serial or d == MAX_DEPTH:
            out.append((s, e, d))
            return
        k = s
        while k < e:
            p = prefix_key(keys[k], d + 1)
            j = k
            while j < e and prefix_key(keys[j], d + 1) == p:
                j += 1
            divide(k, j, d + 1)
            k = j

    if keys:
        divide(0, len(keys), 0)
    return out


def leaves_in_block(block_keys, n_leaf: int, d_root: int):
    """The leaves of one block, read off its own sorted keys as Sec. 2.3.1 does
    for the whole set, with the leaf depth of eq. 2:
        D_k = max(minDepth(k, k-1), minDepth(k, k + n_leaf), d_root)
    where the two neighbours count only inside the block (capped at depth 21).
    Returns [(depth, key, first, count)] with first relative to the block."""
    keys = [int(x) for x in block_keys]
    n = len(keys)
    out = []
    k = 0
    while k < n:
        left = min_depth(keys[k - 1], keys[k]) if k > 0 else 0
        right = min_depth(keys[k], keys[k + n_leaf]) if k + n_leaf < n else 0
        depth = min(max(left, right, d_root), MAX_DEPTH)
        prefix = prefix_key(keys[k], depth)
        stop = k + 1
        while stop < n and prefix_key(keys[stop], depth) == prefix:
            stop += 1
        out.append((depth, prefix, k, stop - k))
        k = stop
    return out


def subtree_build(sorted_keys, n_leaf: int, n_serial: int):
    """All cells by the subtree-rooted method: every block builds its own leaves
    (eq. 2) and its parents up to its root, independently; the cells above the
    block roots are then built from the roots, bottom-up (Sec. 2.3.3).
    Returns {(depth, key): dict(first, count, children, leaf)} like
    parents_bottom_up."""
    cells = {}
    roots = []
    for s, e, d_root in subtree_blocks(sorted_keys, n_serial):
        leaves = [(d, key, s + f, c) for d, key, f, c in
                  leaves_in_block(sorted_keys[s:e], n_leaf, d_root)]
        sub = parents_bottom_up(leaves)
        # the block's cells stop at its root
        for (d, key), cl in sub.items():
            if d >= d_root:
                cells[(d, key)] = cl
        root_key = prefix_key(int(sorted_keys[s]), d_root)
        roots.append((d_root, root_key, s, e - s))
    # upper cells: the block roots play the part of leaves for the cells above
    upper = parents_bottom_up(roots)
    for (d, key), cl in upper.items():
        if not cl["leaf"]:
            cells[(d, key)] = cl
    return cells
