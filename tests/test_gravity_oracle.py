"""Pins of the CPU gravity references (Sec. 2.1), against physics and closed
forms rather than against themselves:

* direct summation: the two-body force in closed form; Newton's third law
  (sum of m a vanishes); the potential of a Plummer sphere, -M / sqrt(r^2 + a^2);
* tree walk: with theta = 0 every cell is opened and the walk is the direct sum;
  the error against the direct sum shrinks with theta; the quadrupole term makes
  the forces more accurate than the monopole alone (the physical check of the
  moments the tree build computes).
"""
import numpy as np
import pytest

import oracle
from paper_2312_06102_amd import datagen as dg


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_direct_two_body_closed_form():
    pos = np.array([[0.25, 0.5, 0.5], [0.75, 0.5, 0.625]], np.float32)
    mass = np.array([0.5, 0.25], np.float32)
    acc = oracle.direct_forces(pos, mass, eps=0.0)
    d = pos[0].astype(np.float64) - pos[1].astype(np.float64)
    r = np.sqrt(d @ d)
    np.testing.assert_allclose(acc[0, :3], -0.25 * d / r ** 3, rtol=1e-15)
    np.testing.assert_allclose(acc[1, :3], 0.5 * d / r ** 3, rtol=1e-15)
    np.testing.assert_allclose(acc[:, 3], [-0.25 / r, -0.5 / r], rtol=1e-15)


def test_direct_newton_third_law():
    pos, mass = dg.plummer(3000, seed=5)
    acc = oracle.direct_forces(pos, mass, eps=1e-4)
    m = mass.astype(np.float64)[:, None]
    total = (m * acc[:, :3]).sum(0)
    scale = (m * np.abs(acc[:, :3])).sum(0)
    assert np.all(np.abs(total) <= 1e-12 * scale)


def test_direct_plummer_potential():
    """A Plummer sphere of scale radius a: phi(r) = -M / sqrt(r^2 + a^2)."""
    rng = _rng(9)
    n, a = 8192, 0.005
    r = dg.plummer_radii(rng, n, rmax=90.0)
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    pos = (0.5 + a * r[:, None] * v).astype(np.float32)
    mass = np.full(n, 1.0 / n, np.float32)
    acc = oracle.direct_forces(pos, mass, eps=1e-5)
    rr = np.linalg.norm(pos.astype(np.float64) - 0.5, axis=1)
    want = -1.0 / np.sqrt(rr ** 2 + a ** 2)
    rel = np.abs(acc[:, 3] - want) / np.abs(want)
    assert np.median(rel) < 0.02, np.median(rel)


def _walk_errors(pos, mass, tree, direct_sorted, theta, quad, n_crit=256):
    w, st = oracle.walk_forces(pos, mass, tree, theta=theta, n_crit=n_crit, eps=1e-4,
                               quadrupole=quad)
    err = np.linalg.norm(w[:, :3] - direct_sorted[:, :3], axis=1) / np.linalg.norm(
        direct_sorted[:, :3], axis=1)
    return w, st, err


@pytest.fixture(scope="module")
def plummer_case():
    pos, mass = dg.plummer(6000, seed=13)
    tree = oracle.build(pos, mass, 10)
    direct = oracle.direct_forces(pos, mass, eps=1e-4)[tree["perm"]]
    return pos, mass, tree, direct


def test_walk_theta_zero_is_direct_sum(plummer_case):
    pos, mass, tree, direct = plummer_case
    for quad in (False, True):
        w, st, _ = _walk_errors(pos, mass, tree, direct, 0.0, quad)
        dev = np.linalg.norm(w[:, :3] - direct[:, :3], axis=1)
        assert np.all(dev <= 1e-12 * w[:, 4])
        assert np.all(np.abs(w[:, 3] - direct[:, 3]) <= 1e-12 * np.abs(direct[:, 3]))
        n = pos.shape[0]
        assert st["interactions"] == n * (n - 1)


def test_walk_error_shrinks_with_theta_and_quadrupole_helps(plummer_case):
    pos, mass, tree, direct = plummer_case
    med = {}
    for theta in (0.3, 0.5, 0.75):
        for quad in (False, True):
            med[theta, quad] = np.median(_walk_errors(pos, mass, tree, direct, theta, quad)[2])
    for quad in (False, True):
        assert med[0.3, quad] < med[0.5, quad] < med[0.75, quad]
    for theta in (0.3, 0.5, 0.75):
        assert med[theta, True] < med[theta, False], (theta, med)
    assert med[0.5, True] <= 0.5 * med[0.5, False], med
    assert med[0.5, False] < 2e-3, med


def test_walk_groups_and_single_group(plummer_case):
    pos, mass, tree, direct = plummer_case
    # every particle is in exactly one group; n_crit >= N makes the root the only group
    _, st = oracle.walk_forces(pos, mass, tree, theta=0.75, n_crit=pos.shape[0], eps=1e-4)
    assert st["groups"] == 1
    _, st1 = oracle.walk_forces(pos, mass, tree, theta=0.75, n_crit=1, eps=1e-4)
    assert st1["groups"] == int((tree["child_ptr"][:, 0] < 0).sum())  # every leaf


def dumbbell_case():
    """Two equal masses 0.01 apart near (0.2, 0.2, 0.2) and a test particle
    near (0.8, 0.7, 0.9): with n_leaf = 1 the test particle's group accepts the
    depth-2 cell holding the pair.  For equal masses the octupole vanishes, so
    the expansion to the quadrupole is exact to O((s/R)^4) ~ 1e-8, while the
    monopole alone is off by O((s/R)^2) ~ 1e-4."""
    u = np.array([1.0, 2.0, 3.0]) / np.sqrt(14.0)
    c = np.array([0.2, 0.2, 0.2])
    pos = np.array([c + 0.005 * u, c - 0.005 * u, [0.8, 0.7, 0.9]], np.float32)
    mass = np.array([0.5, 0.5, 0.25], np.float32)
    return pos, mass


def dumbbell_errors(lib=None):
    pos, mass = dumbbell_case()
    tree = oracle.build(pos, mass, 1, lib=lib)
    direct = oracle.direct_forces(pos, mass, lib=lib)[tree["perm"]]
    k = int(np.nonzero(tree["perm"] == 2)[0][0])  # the test particle's sorted slot
    out = {}
    for quad in (False, True):
        w, _ = oracle.walk_forces(pos, mass, tree, theta=0.75, n_crit=1, quadrupole=quad, lib=lib)
        out[quad] = (np.linalg.norm(w[k, :3] - direct[k, :3]) / np.linalg.norm(direct[k, :3]),
                     abs(w[k, 3] - direct[k, 3]) / abs(direct[k, 3]))
    return out


def test_walk_quadrupole_of_a_distant_dumbbell():
    e = dumbbell_errors()
    assert e[True][0] < 1e-7 and e[True][1] < 1e-7, e
    assert e[False][0] > 1e-5 and e[False][1] > 1e-5, e  # the cell was accepted, not opened


def test_direct_subset_matches_all_pairs(plummer_case):
    pos, mass, _, _ = plummer_case
    full = oracle.direct_forces(pos, mass, eps=1e-4)
    idx = np.array([0, 17, 2999, 5999])
    sub = oracle.direct_forces_at(pos, mass, idx, eps=1e-4)
    assert np.array_equal(sub, full[idx])
