"""Seeded synthetic particle sets.

This module only draws inputs; it holds none of the tree method's arithmetic, and
both the HIP path's tests and the CPU oracle's tests take their inputs from here.

The paper measures on NEMO Plummer spheres and exponential disks (Sec. 3); those
files are not available, so the sets below are drawn from the same analytic
distributions:

* ``uniform``   -- iid in the unit cube, equal masses.
* ``plummer``   -- Plummer sphere (scale radius 1) truncated at r = 50, then
                  normalised into the unit cube.
* ``clustered`` -- cosmology-like: 70 % of the particles in NFW halos whose
                  particle counts follow dN/dM ~ M^-1.9, 30 % uniform background,
                  periodic unit box.
* ``lognormal_masses`` -- m = exp(Z), Z ~ N(0, 1), normalised to sum 1.
* ``batched_sizes`` / ``batched_plummer`` -- many independent Plummer sets with
                  log-uniform sizes.
* ``exponential_disk`` -- thin disk, surface density ~ exp(-R/h) truncated at
                  R = 10 h, vertical density ~ sech^2(z/z0) with z0 = 0.1 h,
                  normalised into the unit cube.
* ``plummer_sim`` / ``disk_sim`` -- the same two distributions with velocities
                  in equilibrium (G = 1, total mass 1, the unit-cube frame), for
                  multi-step runs: Plummer speeds by the rejection method of
                  Aarseth, Henon & Wielen (1974); disk particles on circular
                  orbits (Freeman's exponential-disk rotation curve) with a 10 %
                  velocity dispersion.

Every generator draws in FP64 with numpy's PCG64 and casts to FP32 last.
"""
from __future__ import annotations

import math

import numpy as np

F32_BELOW_ONE = np.float32(np.nextafter(np.float32(1.0), np.float32(0.0)))


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def equal_masses(n: int) -> np.ndarray:
    """1/N each (exact when N is a power of two)."""
    return np.full(n, np.float32(1.0 / max(n, 1)), dtype=np.float32)


def uniform(n: int, seed: int = 1):
    """N iid points in [0,1)^3 (FP32), equal masses."""
    rng = _rng(seed)
    pos = rng.random((n, 3), dtype=np.float32)
    return pos, equal_masses(n)


def _isotropic(rng, n):
    v = rng.standard_normal((n, 3))
    norm = np.sqrt(np.einsum("ij,ij->i", v, v))
    norm[norm == 0] = 1.0
    return v / norm[:, None]


def _unit_cube_map(x: np.ndarray):
    """Affine map of a point cloud into [0,1)^3: centre of the bounding box to 1/2,
    largest extent (times 1 + 2^-20) to 1; cast to FP32 and clamp below 1.
    Returns (points, scale S): lengths shrink by 1/S."""
    if x.shape[0] == 0:
        return x.astype(np.float32), 1.0
    mn = x.min(axis=0)
    mx = x.max(axis=0)
    centre = 0.5 * (mn + mx)
    s = float((mx - mn).max()) * (1.0 + 2.0 ** -20)
    if s == 0.0:
        s = 1.0
    y = 0.5 + (x - centre) / s
    y = y.astype(np.float32)
    np.clip(y, np.float32(0.0), F32_BELOW_ONE, out=y)
    return y, s


def _to_unit_cube(x: np.ndarray) -> np.ndarray:
    return _unit_cube_map(x)[0]


def plummer_radii(rng, n: int, rmax: float = 50.0) -> np.ndarray:
    """Radii of a Plummer sphere with scale radius 1: the enclosed mass fraction is
    M(r) = r^3 (1 + r^2)^-3/2; invert it for u ~ U(0, M(rmax))."""
    mmax = rmax ** 3 * (1.0 + rmax ** 2) ** -1.5
    u = rng.random(n) * mmax
    u = np.maximum(u, np.finfo(np.float64).tiny)
    return (u ** (-2.0 / 3.0) - 1.0) ** -0.5


def plummer(n: int, seed: int = 2, masses: str = "equal"):
    """Plummer sphere (scale radius 1, truncated at 50) normalised into the unit cube."""
    rng = _rng(seed)
    r = plummer_radii(rng, n)
    x = r[:, None] * _isotropic(rng, n)
    pos = _to_unit_cube(x)
    mass = equal_masses(n) if masses == "equal" else lognormal_masses(n, seed + 1000)
    return pos, mass


def _plummer_speeds(rng, r: np.ndarray) -> np.ndarray:
    """Speeds of a Plummer sphere (G = M = a = 1) at radii r: v = q v_esc with
    v_esc = sqrt(2) (1 + r^2)^-1/4 and q drawn from g(q) ~ q^2 (1 - q^2)^7/2 by
    rejection (Aarseth, Henon & Wielen 1974)."""
    n = r.shape[0]
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        x1 = rng.random(todo.size)
        x2 = rng.random(todo.size)
        ok = 0.1 * x2 < x1 * x1 * (1.0 - x1 * x1) ** 3.5
        q[todo[ok]] = x1[ok]
        todo = todo[~ok]
    return q * np.sqrt(2.0) * (1.0 + r * r) ** -0.25


def _scaled_velocities(v: np.ndarray, s: float) -> np.ndarray:
    """Velocities in the unit-cube frame: with G and the total mass fixed,
    shrinking lengths by 1/S speeds orbits up by sqrt(S)."""
    return (v * math.sqrt(s)).astype(np.float32)


def plummer_sim(n: int, seed: int = 12):
    """Plummer sphere in equilibrium: (pos, vel, mass) in the unit-cube frame,
    G = 1, total mass 1 (masses 1/N)."""
    rng = _rng(seed)
    r = plummer_radii(rng, n)
    x = r[:, None] * _isotropic(rng, n)
    v = _plummer_speeds(rng, r)[:, None] * _isotropic(rng, n)
    pos, s = _unit_cube_map(x)
    return pos, _scaled_velocities(v, s), equal_masses(n)


def _disk_radii(rng, n: int, rmax: float = 10.0) -> np.ndarray:
    """Radii of an exponential disk of scale length 1 truncated at rmax: the
    enclosed mass fraction 1 - (1 + R) e^-R inverted by bisection."""
    def frac(R):
        return 1.0 - (1.0 + R) * np.exp(-R)
    u = rng.random(n) * frac(rmax)
    lo = np.zeros(n)
    hi = np.full(n, rmax)
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        below = frac(mid) < u
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    return 0.5 * (lo + hi)


def _disk_positions(rng, n: int, z0: float = 0.1, rmax: float = 10.0):
    R = _disk_radii(rng, n, rmax)
    phi = rng.random(n) * (2.0 * math.pi)
    z = z0 * np.arctanh(np.clip(2.0 * rng.random(n) - 1.0, -1.0 + 1e-15, 1.0 - 1e-15))
    x = np.stack([R * np.cos(phi), R * np.sin(phi), z], axis=1)
    return x, R, phi


def exponential_disk(n: int, seed: int = 6, z0: float = 0.1):
    """Thin exponential disk (scale length 1, sech^2 scale height z0, truncated
    at R = 10) normalised into the unit cube; equal masses."""
    rng = _rng(seed)
    x, _, _ = _disk_positions(rng, n, z0)
    return _to_unit_cube(x), equal_masses(n)


def disk_sim(n: int, seed: int = 13, z0: float = 0.1, sigma: float = 0.1):
    """Exponential disk with velocities: (pos, vel, mass) in the unit-cube frame,
    G = 1, disk mass 1.  Circular speed of the (untruncated) razor-thin disk,
    v_c^2 = 2 y^2 [I0(y) K0(y) - I1(y) K1(y)] with y = R/2 (Freeman 1970), plus
    isotropic Gaussian motions of sigma * v_c per axis."""
    from scipy import special
    rng = _rng(seed)
    x, R, phi = _disk_positions(rng, n, z0)
    y = np.maximum(0.5 * R, 1e-8)
    vc = np.sqrt(np.maximum(2.0 * y * y * (special.i0(y) * special.k0(y)
                                           - special.i1(y) * special.k1(y)), 0.0))
    v = np.stack([-vc * np.sin(phi), vc * np.cos(phi), np.zeros(n)], axis=1)
    v += sigma * vc[:, None] * rng.standard_normal((n, 3))
    pos, s = _unit_cube_map(x)
    return pos, _scaled_velocities(v, s), equal_masses(n)


def _halo_counts(rng, n_halo_particles: int, n_halos: int, mmin=1e2, mmax=1e6, slope=1.9):
    """Halo particle counts: n_halos draws from dN/dM ~ M^-slope on [mmin, mmax] by
    inverse CDF, rescaled by one common factor so that they sum to
    n_halo_particles (largest-remainder rounding)."""
    u = rng.random(n_halos)
    a = 1.0 - slope
    m = (mmin ** a + u * (mmax ** a - mmin ** a)) ** (1.0 / a)
    scaled = m * (n_halo_particles / m.sum())
    base = np.floor(scaled).astype(np.int64)
    rem = n_halo_particles - int(base.sum())
    if rem > 0:
        order = np.argsort(-(scaled - base), kind="stable")
        base[order[:rem]] += 1
    return base


def _nfw_mu(x):
    return np.log1p(x) - x / (1.0 + x)


def _nfw_radii(rng, n: int, c: float, r_s: float) -> np.ndarray:
    """NFW radii truncated at r = c*r_s: solve mu(x) = u*mu(c) by bisection."""
    target = rng.random(n) * _nfw_mu(c)
    lo = np.zeros(n)
    hi = np.full(n, c)
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        f = _nfw_mu(mid) < target
        lo = np.where(f, mid, lo)
        hi = np.where(f, hi, mid)
    return 0.5 * (lo + hi) * r_s


def clustered(n: int, seed: int = 3, n_halos: int = 2000, halo_fraction: float = 0.7,
              masses: str = "equal"):
    """Cosmology-like clustered set in the periodic unit box."""
    rng = _rng(seed)
    n_h = int(round(halo_fraction * n))
    n_halos = max(1, min(n_halos, n_h)) if n_h > 0 else 0
    counts = _halo_counts(rng, n_h, n_halos) if n_halos else np.zeros(0, np.int64)
    parts = []
    for nh in counts:
        nh = int(nh)
        centre = rng.random(3)
        conc = rng.uniform(5.0, 15.0)
        if nh == 0:
            continue
        r200 = (3.0 * nh / (4.0 * math.pi * 200.0 * n)) ** (1.0 / 3.0)
        r = _nfw_radii(rng, nh, conc, r200 / conc)
        parts.append(centre + r[:, None] * _isotropic(rng, nh))
    parts.append(rng.random((n - n_h, 3)))
    x = np.concatenate(parts, axis=0) if parts else np.zeros((0, 3))
    x = np.mod(x, 1.0)
    pos = x.astype(np.float32)
    pos[pos >= np.float32(1.0)] = np.float32(0.0)
    # shuffle so that the input order carries no spatial structure
    pos = pos[rng.permutation(n)]
    mass = equal_masses(n) if masses == "equal" else lognormal_masses(n, seed + 1000)
    return pos, mass


def lognormal_masses(n: int, seed: int = 5, sigma: float = 1.0) -> np.ndarray:
    """m = exp(Z), Z ~ N(0, sigma^2), normalised to sum 1 (in FP64, then cast)."""
    rng = _rng(seed)
    m = np.exp(sigma * rng.standard_normal(n))
    m /= m.sum()
    out = m.astype(np.float32)
    out[out <= 0] = np.float32(np.finfo(np.float32).tiny)
    return out


def batched_sizes(n_sets: int = 4096, lo: int = 256, hi: int = 262144, seed: int = 4):
    """Set sizes floor(exp(U(ln lo, ln hi)))."""
    rng = _rng(seed)
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), n_sets))).astype(np.int64)


def batched_plummer(sizes, seed: int = 4):
    """Concatenated independent Plummer sets, each normalised into its own unit cube,
    masses 1/n_b.  Returns (pos [sum,3], mass [sum], offsets [B+1])."""
    sizes = np.asarray(sizes, dtype=np.int64)
    children = np.random.SeedSequence(seed).spawn(len(sizes))
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    pos = np.empty((int(offsets[-1]), 3), dtype=np.float32)
    mass = np.empty(int(offsets[-1]), dtype=np.float32)
    for b, (nb, ss) in enumerate(zip(sizes, children)):
        if nb == 0:
            continue
        rng = np.random.Generator(np.random.PCG64(ss))
        r = plummer_radii(rng, int(nb))
        x = r[:, None] * _isotropic(rng, int(nb))
        pos[offsets[b]:offsets[b + 1]] = _to_unit_cube(x)
        mass[offsets[b]:offsets[b + 1]] = np.float32(1.0 / nb)
    return pos, mass, offsets


# Named workloads -------------------------------------------------------------

def workload(name: str, n: int | None = None):
    """(pos, mass, n_leaf) for a named workload.

    uniform64k   : N = 65,536 uniform, n_leaf 16
    plummer16m   : N = 2^24 Plummer, n_leaf 16
    clustered64m : N = 2^26 clustered, n_leaf 8
    mixed16m     : N = 2^24 clustered with log-normal masses, n_leaf 8
    disk16m      : N = 2^24 exponential disk, n_leaf 16
    """
    if name == "uniform64k":
        p, m = uniform(n or 65536, seed=1)
        return p, m, 16
    if name == "plummer16m":
        p, m = plummer(n or (1 << 24), seed=2)
        return p, m, 16
    if name == "clustered64m":
        p, m = clustered(n or (1 << 26), seed=3)
        return p, m, 8
    if name == "mixed16m":
        p, m = clustered(n or (1 << 24), seed=5, masses="lognormal")
        return p, m, 8
    if name == "disk16m":
        p, m = exponential_disk(n or (1 << 24), seed=6)
        return p, m, 16
    raise KeyError(name)
