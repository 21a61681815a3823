"""The subtree-rooted cell build (TB_SUBTREES, Sec. 2.3.3 with eq. 2) against
the CPU oracle, through the C ABI.

The flag changes how the cells are built (blocks of at most 2048 particles
built one per workgroup from their roots' depth, the cells above the blocks
last), not what they are: perm, keys and structure bit-identical to the oracle,
FP64 moments within the same 1e-12 per-cell relative measures, mixed-precision
moments within 1e-6.  The cases cover ragged sizes around the block size,
n_leaf from 1 to 1024, saturated depth-21 leaves, duplicate-heavy and
clustered inputs, boxes that do not hold every point, and batches of uneven
sets.
"""
import numpy as np
import pytest

import oracle
from paper_2312_06102_amd import datagen as dg
from test_gpu_batched import batch_build, check_against_oracle, check_offsets, uneven_sizes
from test_gpu_parity import (FP64_TOL, MIXED_TOL, compare_structure, full_parity, gpu_build,
                             moment_errors)

pytestmark = pytest.mark.gpu


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.mark.parametrize("n", [1, 2, 17, 2047, 2048, 2049, 4097, 10007, 100003])
def test_uniform_sizes(n):
    rng = _rng(100 + n)
    pos = rng.random((n, 3), dtype=np.float32)
    mass = (rng.random(n) + 0.1).astype(np.float32)
    full_parity(pos, mass, 16, subtrees=True)


@pytest.mark.parametrize("n_leaf", [1, 2, 8, 33, 64, 1024])
def test_n_leaf_values(n_leaf):
    pos, mass = dg.plummer(30000, seed=8)
    full_parity(pos, mass, n_leaf, subtrees=True)


def test_plummer_200k():
    pos, mass = dg.plummer(200000, seed=22)
    full_parity(pos, mass, 16, subtrees=True)


def test_clustered_lognormal():
    pos, mass = dg.clustered(150000, seed=23, n_halos=150, masses="lognormal")
    full_parity(pos, mass, 8, subtrees=True)


def test_coincident_points_depth21_leaf():
    """More identical points than the block holds: the one saturated depth-21
    leaf spans several blocks' worth of particles."""
    pos = np.tile(np.array([[0.3, 0.7, 0.1]], np.float32), (5000, 1))
    mass = np.full(5000, 2.0 ** -12, np.float32)
    g, o = full_parity(pos, mass, 8, subtrees=True)
    assert g["n_cells"] == 22 and g["cell_count"][21] == 5000


def test_duplicates_and_pairs():
    rng = _rng(24)
    base = rng.random((300, 3), dtype=np.float32)
    pos = np.repeat(base, rng.integers(1, 40, 300), axis=0)
    pairs = np.repeat((rng.random((3000, 3)) * 0.25).astype(np.float32), 2, axis=0)
    pos = np.concatenate([pos, pairs, rng.random((12000, 3), dtype=np.float32)])
    pos = pos[rng.permutation(pos.shape[0])]
    mass = (rng.random(pos.shape[0]) + 0.5).astype(np.float32)
    full_parity(pos, mass, 1, subtrees=True)
    full_parity(pos, mass, 4, subtrees=True)


def test_complete_lattice():
    g1 = (np.arange(32) + 0.5) / 32
    pos = np.stack(np.meshgrid(g1, g1, g1, indexing="ij"), -1).reshape(-1, 3).astype(np.float32)
    g, o = full_parity(pos, np.ones(pos.shape[0], np.float32), 1, subtrees=True)
    for d in range(6):
        assert g["level_offset"][d + 1] - g["level_offset"][d] == 8 ** d


def test_points_outside_box_and_auto_box():
    rng = _rng(25)
    pos = (rng.random((20000, 3)) * 1.4 - 0.2).astype(np.float32)
    full_parity(pos, np.ones(20000, np.float32), 16, extent=True, subtrees=True)
    pos = (rng.standard_normal((40000, 3)) * 3.0 + 7.0).astype(np.float32)
    lo, side = oracle.auto_box(pos)
    full_parity(pos, np.ones(40000, np.float32), 16, lo=lo, side=side, box="auto",
                subtrees=True)


def test_mixed_precision():
    pos, mass = dg.clustered(100000, seed=26, n_halos=100, masses="lognormal")
    o = oracle.build(pos, mass, 8)
    g = gpu_build(pos, mass, 8, precision="mixed", subtrees=True)
    compare_structure(g, o)
    e = moment_errors(g["com"].astype(np.float64), g["quad"].astype(np.float64), o["com"],
                      o["quad"], o["cell_level"])
    assert max(e) <= MIXED_TOL, e


def test_both_paths_same_tree():
    """The flag leaves the tree as it is: both paths give the same structure and
    FP64 moments within rounding of each other."""
    pos, mass = dg.plummer(120000, seed=27)
    a = gpu_build(pos, mass, 16)
    b = gpu_build(pos, mass, 16, subtrees=True)
    compare_structure(a, b)
    e = moment_errors(b["com"], b["quad"], a["com"], a["quad"], a["cell_level"])
    assert max(e) <= FP64_TOL, e


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_uneven_sets(precision):
    sizes = uneven_sizes()
    pos, mass, offsets = dg.batched_plummer(sizes, seed=28)
    g = batch_build(pos, mass, offsets, 16, precision=precision, subtrees=True)
    check_offsets(g, offsets)
    check_against_oracle(pos, mass, offsets, 16, g, range(len(sizes)),
                         tol=FP64_TOL if precision == "fp64" else MIXED_TOL)


def test_batched_thousands_of_sets():
    rng = _rng(29)
    sizes = rng.integers(0, 600, 3000)
    pos, mass, offsets = dg.batched_plummer(sizes, seed=29)
    g = batch_build(pos, mass, offsets, 8, subtrees=True)
    check_offsets(g, offsets)
    check_against_oracle(pos, mass, offsets, 8, g, rng.choice(len(sizes), 60, replace=False))
