"""The multi-step inputs are in equilibrium and have the intended shapes.

These check the seeded generators (they hold none of the tree method): a
Plummer sphere with Aarseth-Henon-Wielen speeds and a rotating exponential
disk, both in virial balance (2T/|W| near 1, W from the oracle's direct sum);
the disk's surface density falls off as exp(-R/h) and it is thin.
"""
import numpy as np

import oracle
from paper_2312_06102_amd import datagen as dg


def _virial(pos, vel, mass):
    d = oracle.direct_forces(pos, mass, eps=0.0)
    w = 0.5 * np.sum(mass.astype(np.float64) * d[:, 3])
    t = 0.5 * np.sum(mass.astype(np.float64) * (vel.astype(np.float64) ** 2).sum(1))
    return 2.0 * t / abs(w)


def test_plummer_in_virial_balance():
    pos, vel, mass = dg.plummer_sim(4096)
    assert pos.dtype == vel.dtype == mass.dtype == np.float32
    assert pos.min() >= 0.0 and pos.max() < 1.0
    assert abs(_virial(pos, vel, mass) - 1.0) < 0.05
    # isotropic: no net rotation, equal dispersion along the axes
    s = vel.astype(np.float64).std(0)
    assert s.max() / s.min() < 1.1


def test_disk_shape_and_rotation():
    pos, vel, mass = dg.disk_sim(20000)
    c = 0.5 * (pos.min(0) + pos.max(0))
    x = pos.astype(np.float64) - c
    R = np.hypot(x[:, 0], x[:, 1])
    h = np.median(R) / 1.678  # median radius of an exponential disk is 1.678 h
    # surface density ~ exp(-R/h): fit the slope of ln(N(R) / R) between h and 5h
    edges = np.linspace(h, 5 * h, 17)
    cnt, _ = np.histogram(R, edges)
    mid = 0.5 * (edges[1:] + edges[:-1])
    slope = np.polyfit(mid, np.log(cnt / mid), 1)[0]
    assert abs(slope * h + 1.0) < 0.1
    # thin: vertical spread about a tenth of the scale length
    assert 0.05 < np.std(x[:, 2]) / h < 0.25
    # rotating: tangential velocity dominates
    vt = (x[:, 0] * vel[:, 1] - x[:, 1] * vel[:, 0]) / np.maximum(R, 1e-12)
    assert np.mean(vt) > 3.0 * np.std(vel[:, 2])
    assert abs(_virial(pos[:4096], vel[:4096], mass[:4096] * (20000 / 4096)) - 1.0) < 0.2
