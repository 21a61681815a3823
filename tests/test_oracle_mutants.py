"""The oracle's pins catch plausible mistakes.

Each case copies ``oracle/tb_oracle.c``, plants one mistake by text substitution
(a swapped axis, an off-by-one split threshold, a wrong sign, a dropped term, a
wrong bit index, a wrong tie order, a rounding instead of a floor), compiles the
copy with gcc and runs the pin checks against it: at least one must fail, and
all of them must pass on the unmodified source.
"""
import os

import numpy as np
import pytest

import oracle
import treecheck as tc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

MUTANTS = {
    "axis_order": ("k = (k << 1) | ((qx >> b) & 1u);\n    k = (k << 1) | ((qy >> b) & 1u);",
                   "k = (k << 1) | ((qy >> b) & 1u);\n    k = (k << 1) | ((qx >> b) & 1u);"),
    "split_threshold": ("if (t->v[node].cnt <= t->n_leaf ||", "if (t->v[node].cnt < t->n_leaf ||"),
    "octant_bit": ("int b = TBO_MAX_DEPTH - 1 - level;", "int b = TBO_MAX_DEPTH - 2 - level;"),
    "quad_sign": ("nsum_add(&s2[0], m * (3.0 * r[0] * r[0] - r2));",
                  "nsum_add(&s2[0], m * (3.0 * r[0] * r[0] + r2));"),
    "quad_offdiag": ("nsum_add(&s2[4], m * (3.0 * r[1] * r[2]));",
                     "nsum_add(&s2[4], m * (3.0 * r[1] * r[0]));"),
    "drop_centre": ("double r = ((double)pos[3 * (int64_t)p + a] - lo[a]) - off[a];",
                    "double r = ((double)pos[3 * (int64_t)p + a] - lo[a]);"),
    "quad_about_centre": ("- off[a]) - c[a];", "- off[a]);"),
    "tie_order": ("return (x->idx > y->idx) - (x->idx < y->idx);\n}\n\nstatic const uint64_t",
                  "return (x->idx < y->idx) - (x->idx > y->idx);\n}\n\nstatic const uint64_t"),
    "round_not_floor": ("return (uint32_t)floor(t);", "return (uint32_t)floor(t + 0.5);"),
    "centre_half": ("off[0] = ((double)ijk[0] + 0.5) * h;", "off[0] = ((double)ijk[0]) * h;"),
    "depth_cap": ("#define TBO_MAX_DEPTH 21", "#define TBO_MAX_DEPTH 20"),
    # the single-cell entry point used by the sampled full-size checks
    "cell_moments_first_count": (
        "cell_moments(pos, mass, lo, side, perm, first, count, key, level, 0, com_out, quad_out);",
        "cell_moments(pos, mass, lo, side, perm, count, first, key, level, 0, com_out, quad_out);"),
    "cell_moments_frame": (
        "cell_moments(pos, mass, lo, side, perm, first, count, key, level, 0, com_out, quad_out);",
        "cell_moments(pos, mass, lo, side, perm, first, count, key >> 3, level - 1, 0, com_out,"
        " quad_out);"),
    # Peano-Hilbert keys
    "hilbert_gray_step": ("  X[1] ^= X[0];\n  X[2] ^= X[1];\n  t = 0;", "  X[2] ^= X[1];\n  t = 0;"),
    "hilbert_last_level": ("for (Q = 1u << (bits - 1); Q > 1u; Q >>= 1) {\n    P = Q - 1u;",
                           "for (Q = 1u << (bits - 1); Q > 2u; Q >>= 1) {\n    P = Q - 1u;"),
    "hilbert_digit_order": ("h = (h << 1) | ((X[i] >> b) & 1u);",
                            "h = (h << 1) | ((X[2 - i] >> b) & 1u);"),
    "hilbert_decode_gray": ("    X[0] ^= t;\n    for (Q = 2u;", "    for (Q = 2u;"),
    "hilbert_child_key": ("uint64_t key = t->keys[p] >> (3 * (TBO_MAX_DEPTH - lvl));",
                          "uint64_t key = (t->v[node].key << 3) | (uint64_t)oct;"),
}


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _pin_checks(lib):
    """Run a compact set of the pins against ``lib``; return the names that fail."""
    failures = []

    def check(name, fn):
        try:
            fn()
        except Exception:  # a failed pin, or the planted bug crashing the checker
            failures.append(name)

    def hand_keys():
        rows = [ln.split() for ln in open(os.path.join(GOLDEN, "hand_keys.txt"))
                if ln.strip() and not ln.startswith("#")]
        pos = np.array([[float(r[0]), float(r[1]), float(r[2])] for r in rows], np.float32)
        _, k = oracle.keys(pos, lib=lib)
        assert np.array_equal(k, np.array([int(r[3]) for r in rows], np.uint64))

    def set_definition():
        rng = _rng(11)
        base = rng.random((5, 3), dtype=np.float32)
        for pos, nl in [(rng.random((120, 3), dtype=np.float32), 4),
                        (np.repeat(base, [1, 2, 7, 9, 3], axis=0), 4)]:
            t = oracle.build(pos, np.ones(pos.shape[0], np.float32), nl, moments=False, lib=lib)
            g = tc.geometric_tree(pos, nl)
            assert t["n_cells"] == len(g["cells"])
            assert np.array_equal(t["perm"], g["perm"])
            for c, cl in enumerate(g["cells"]):
                assert int(t["cell_key"][c]) == cl["key"]
                f, n = int(t["cell_first"][c]), int(t["cell_count"][c])
                assert list(t["perm"][f:f + n]) == cl["members"]

    def coincident():
        pos = np.tile(np.array([[0.3, 0.7, 0.1]], np.float32), (40, 1))
        t = oracle.build(pos, np.ones(40, np.float32), 8, lib=lib)
        assert t["n_cells"] == 22 and np.all(t["cell_count"] == 40)

    def exact_moments():
        rng = _rng(201)
        pos = rng.random((40, 3), dtype=np.float32)
        mass = (rng.random(40) + 0.1).astype(np.float32)
        t = oracle.build(pos, mass, 3, lib=lib)
        for c in range(t["n_cells"]):
            f, n = int(t["cell_first"][c]), int(t["cell_count"][c])
            lv = int(t["cell_level"][c])
            M, cx, qx = tc.exact_moments(pos, mass, list(t["perm"][f:f + n]), int(t["cell_key"][c]), lv)
            l = 2.0 ** -lv
            assert abs(t["com"][c, 3] - float(M)) <= 1e-15 * float(M)
            assert max(abs(t["com"][c, a] - float(cx[a])) for a in range(3)) <= 1e-15 * l
            assert max(abs(t["quad"][c, i] - float(qx[i])) for i in range(6)) <= 1e-14 * float(M) * l * l

    def cell_moments_wrapper():
        rng = _rng(301)
        lo, side = (-4.0, -4.0, -4.0), 8.0
        pos = (rng.random((50, 3)) * 6.0 - 3.0).astype(np.float32)
        mass = (rng.random(50) + 0.1).astype(np.float32)
        t = oracle.build(pos, mass, 2, lo=lo, side=side, lib=lib)
        for c in range(t["n_cells"]):
            f, n = int(t["cell_first"][c]), int(t["cell_count"][c])
            key, lv = int(t["cell_key"][c]), int(t["cell_level"][c])
            com, quad = oracle.cell_moments(pos, mass, t["perm"], f, n, key, lv, lo=lo, side=side,
                                            lib=lib)
            M, cx, qx = tc.exact_moments(pos, mass, list(t["perm"][f:f + n]), key, lv, lo=lo,
                                         side=side)
            l = side * 2.0 ** -lv
            assert abs(com[3] - float(M)) <= 1e-15 * float(M)
            assert max(abs(com[a] - float(cx[a])) for a in range(3)) <= 1e-15 * l
            assert max(abs(quad[i] - float(qx[i])) for i in range(6)) <= 1e-14 * float(M) * l * l

    def hilbert_curve():
        for bits in (1, 2, 3):
            n = 8 ** bits
            q = oracle.hilbert_decode(np.arange(n, dtype=np.uint64), bits, lib=lib).astype(np.int64)
            assert len({tuple(r) for r in q}) == n and not q[0].any()
            assert np.all(np.abs(np.diff(q, axis=0)).sum(1) == 1)
            h = oracle.hilbert_encode(q.astype(np.uint32), bits, lib=lib)
            assert np.array_equal(h, np.arange(n, dtype=np.uint64))
        q = _rng(401).integers(0, 2 ** 21, (500, 3), dtype=np.uint32)
        h = oracle.hilbert_encode(q, 21, lib=lib)
        for d in (1, 5, 20):
            assert np.array_equal(h >> np.uint64(3 * (21 - d)),
                                  oracle.hilbert_encode(q >> np.uint32(21 - d), d, lib=lib))

    def hilbert_tree():
        rng = _rng(402)
        pos = rng.random((300, 3), dtype=np.float32)
        m = np.ones(300, np.float32)
        tm = oracle.build(pos, m, 4, lib=lib)
        th = oracle.build(pos, m, 4, lib=lib, curve="hilbert")
        assert th["n_cells"] == tm["n_cells"]
        _, k = oracle.keys(pos, lib=lib, curve="hilbert")
        tc.check_invariants(th, k[th["perm"]], 4)
        assert np.allclose(np.sort(th["com"][:, 3]), np.sort(tm["com"][:, 3]), rtol=1e-14)

    check("hand_keys", hand_keys)
    check("hilbert_curve", hilbert_curve)
    check("hilbert_tree", hilbert_tree)
    check("set_definition", set_definition)
    check("coincident", coincident)
    check("exact_moments", exact_moments)
    check("cell_moments_wrapper", cell_moments_wrapper)
    return failures


def _compile(tmp_path, name, src_text):
    src = tmp_path / f"{name}.c"
    src.write_text(src_text)
    out = str(tmp_path / f"lib{name}.so")
    oracle.build_library(str(src), out)
    return oracle.load(out)


def test_unmodified_oracle_passes_pins(tmp_path):
    text = open(oracle.SRC).read()
    lib = _compile(tmp_path, "original", text)
    assert _pin_checks(lib) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    text = open(oracle.SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not found exactly once"
    lib = _compile(tmp_path, name, text.replace(old, new))
    assert _pin_checks(lib), f"no pin caught the planted mistake {name}"


# --------------------------------------------------------------------------
# the gravity references (tb_gravity.c)
# --------------------------------------------------------------------------

GRAVITY_MUTANTS = {
    "quad_sign": ("t[q] += Qr[q] * rinv5 - 2.5 * rQr * r[q] * rinv7;",
                  "t[q] -= Qr[q] * rinv5 - 2.5 * rQr * r[q] * rinv7;"),
    "quad_coefficient": ("t[q] += Qr[q] * rinv5 - 2.5 * rQr * r[q] * rinv7;",
                         "t[q] += Qr[q] * rinv5 - 1.5 * rQr * r[q] * rinv7;"),
    "expansion_about_centre": ("r[q] = xi[q] - (cen[q] + w->com[4 * c + q]);",
                               "r[q] = xi[q] - cen[q];"),
    "open_criterion_side": ("if (l * l < w->theta * w->theta * d2) {",
                            "if (l < w->theta * w->theta * d2) {"),
    "self_term": ("if (j == s) continue;", "if (j == s && 0) continue;"),
    "direct_sign": ("    acc[4 * i + 0] = ax;", "    acc[4 * i + 0] = -ax;"),
}


def _gravity_pins(lib):
    import test_gravity_oracle as tg
    failures = []
    pos, mass = tg.dg.plummer(2500, seed=13)
    tree = oracle.build(pos, mass, 10, lib=lib)
    direct = oracle.direct_forces(pos, mass, eps=1e-4, lib=lib)[tree["perm"]]

    def check(name, fn):
        try:
            fn()
        except Exception:
            failures.append(name)

    def newton():
        acc = oracle.direct_forces(pos, mass, eps=1e-4, lib=lib)
        m = mass.astype(np.float64)[:, None]
        assert np.all(np.abs((m * acc[:, :3]).sum(0)) <= 1e-12 * (m * np.abs(acc[:, :3])).sum(0))
        two = oracle.direct_forces(np.array([[0.25, 0.5, 0.5], [0.75, 0.5, 0.5]], np.float32),
                                   np.array([0.5, 0.25], np.float32), lib=lib)
        assert two[0, 0] > 0 and two[1, 0] < 0  # attraction

    def theta_zero():
        w, _ = oracle.walk_forces(pos, mass, tree, theta=0.0, n_crit=256, eps=1e-4, lib=lib)
        assert np.all(np.linalg.norm(w[:, :3] - direct[:, :3], axis=1) <= 1e-12 * w[:, 4])

    def accuracy():
        med = {}
        for quad in (False, True):
            w, _ = oracle.walk_forces(pos, mass, tree, theta=0.5, n_crit=256, eps=1e-4,
                                      quadrupole=quad, lib=lib)
            err = np.linalg.norm(w[:, :3] - direct[:, :3], axis=1) / np.linalg.norm(
                direct[:, :3], axis=1)
            med[quad] = np.median(err)
        assert med[False] < 2e-3 and med[True] <= 0.5 * med[False], med

    def dumbbell():
        e = tg.dumbbell_errors(lib=lib)
        assert e[True][0] < 1e-7 and e[True][1] < 1e-7 and e[False][0] > 1e-5, e

    check("newton", newton)
    check("theta_zero", theta_zero)
    check("dumbbell", dumbbell)
    check("accuracy", accuracy)
    return failures


def test_unmodified_gravity_passes_pins(tmp_path):
    src = tmp_path / "grav.c"
    src.write_text(open(oracle.GRAVITY_SRC).read())
    out = str(tmp_path / "libgrav.so")
    oracle.build_library(out=out, gravity_src=str(src))
    assert _gravity_pins(oracle.load(out)) == []


@pytest.mark.parametrize("name", sorted(GRAVITY_MUTANTS))
def test_planted_gravity_mistake_is_caught(tmp_path, name):
    old, new = GRAVITY_MUTANTS[name]
    text = open(oracle.GRAVITY_SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not found exactly once"
    src = tmp_path / f"{name}.c"
    src.write_text(text.replace(old, new))
    out = str(tmp_path / f"lib{name}.so")
    oracle.build_library(out=out, gravity_src=str(src))
    assert _gravity_pins(oracle.load(out)), f"no pin caught the planted mistake {name}"
