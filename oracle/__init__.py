"""CPU oracle for the leaf-first oct-tree build -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path
(``paper_2312_06102_amd``) never imports it, and this package imports nothing
from the product path.

The C source ``tb_oracle.c`` is a sequential top-down Barnes-Hut insertion
build (Sec. 2.1) over hashed Morton keys (Sec. 2.2) with direct FP64 moment
sums per cell; see the header comment there for each step and its source.
``tb_leaffirst.c`` is a second CPU reference: the paper's own leaf-first
method (Sec. 2.3, Algorithms 1 and 2) on one thread, moments combined from the
children as cells are created.  ``tb_gravity.c`` holds the gravity references
(Sec. 2.1): O(N^2) direct summation and a sequential Barnes-Hut group walk.
``build_library()`` compiles all three with gcc into ``liboracle.so``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "tb_oracle.c")
LEAF_FIRST_SRC = os.path.join(_HERE, "tb_leaffirst.c")
GRAVITY_SRC = os.path.join(_HERE, "tb_gravity.c")
LIB = os.path.join(_HERE, "liboracle.so")

# Strict IEEE FP64: no contraction into FMA, no fast-math reassociation.
CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wextra", "-Wno-unused-parameter"]

MAX_DEPTH = 21

_lib = None


def build_library(src: str = SRC, out: str = LIB, extra_flags=(), gravity_src: str = GRAVITY_SRC
                  ) -> str:
    """Compile the oracle C source (``src``, normally tb_oracle.c) together with
    the leaf-first reference and the gravity references into a shared library
    (gcc)."""
    cmd = ["gcc", *CFLAGS, *extra_flags, "-o", out + ".tmp", src, LEAF_FIRST_SRC, gravity_src,
           "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(out + ".tmp", out)
    return out


def _bind(lib: ctypes.CDLL) -> ctypes.CDLL:
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.tbo_keys.argtypes = [P, i64, P, ctypes.c_double, P, P]
    lib.tbo_keys.restype = ctypes.c_int
    lib.tbo_keys_curve.argtypes = [P, i64, P, ctypes.c_double, ctypes.c_int, P, P]
    lib.tbo_keys_curve.restype = ctypes.c_int
    lib.tbo_hilbert_encode.argtypes = [P, i64, ctypes.c_int, P]
    lib.tbo_hilbert_encode.restype = None
    lib.tbo_hilbert_decode.argtypes = [P, i64, ctypes.c_int, P]
    lib.tbo_hilbert_decode.restype = None
    lib.tbo_max_cells.argtypes = [i64, ctypes.c_int32]
    lib.tbo_max_cells.restype = i64
    lib.tbo_build.argtypes = [P, P, i64, ctypes.c_int32, P, ctypes.c_double] + [P] * 11
    lib.tbo_build.restype = ctypes.c_int
    lib.tbo_build_timed.argtypes = [P, P, i64, ctypes.c_int32, P, ctypes.c_double] + [P] * 12
    lib.tbo_build_timed.restype = ctypes.c_int
    lib.tbo_build_curve.argtypes = [P, P, i64, ctypes.c_int32, P, ctypes.c_double,
                                    ctypes.c_int] + [P] * 12
    lib.tbo_build_curve.restype = ctypes.c_int
    lib.tbl_build.argtypes = [P, P, i64, ctypes.c_int32, P, ctypes.c_double] + [P] * 11
    lib.tbl_build.restype = ctypes.c_int
    lib.tbo_cell_moments.argtypes = [P, P, P, ctypes.c_double, P, i64, i64,
                                     ctypes.c_uint64, ctypes.c_int, P, P]
    lib.tbo_cell_moments.restype = ctypes.c_int
    lib.tbg_direct.argtypes = [P, P, i64, ctypes.c_double, P]
    lib.tbg_direct.restype = ctypes.c_int
    lib.tbg_direct_subset.argtypes = [P, P, i64, ctypes.c_double, P, i64, P]
    lib.tbg_direct_subset.restype = ctypes.c_int
    lib.tbg_walk_tree.argtypes = [P, P, P, i64] + [P] * 7 + [P, ctypes.c_double, ctypes.c_double,
                                                             ctypes.c_int32, ctypes.c_double,
                                                             ctypes.c_int, P, P]
    lib.tbg_walk_tree.restype = ctypes.c_int
    lib.tbg_walk_tree_curve.argtypes = [P, P, P, i64] + [P] * 7 + [
        P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_double, ctypes.c_int,
        ctypes.c_int, P, P]
    lib.tbg_walk_tree_curve.restype = ctypes.c_int
    lib.tbo_auto_box.argtypes = [P, i64, P, P]
    lib.tbo_auto_box.restype = ctypes.c_int
    return lib


def load(path: Optional[str] = None) -> ctypes.CDLL:
    """Load the oracle library, compiling it first if it is not built yet."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        sources = (SRC, LEAF_FIRST_SRC, GRAVITY_SRC)
        if not os.path.exists(LIB) or any(os.path.getmtime(f) > os.path.getmtime(LIB)
                                           for f in sources):
            build_library()
        _lib = _bind(ctypes.CDLL(LIB))
    return _lib


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle returned error code {code}")
        self.code = code


def _box(lo, side):
    lo = np.ascontiguousarray(np.asarray(lo, dtype=np.float64).reshape(3))
    return lo, float(side)


CURVES = {"morton": 0, "hilbert": 1}


def _curve(curve: str) -> int:
    if curve not in CURVES:
        raise ValueError(f"curve must be one of {sorted(CURVES)}")
    return CURVES[curve]


def keys(pos: np.ndarray, lo=(0.0, 0.0, 0.0), side: float = 1.0, lib=None,
         curve: str = "morton"):
    """Quantised coordinates [N,3] (uint32) and 64-bit keys [N] (uint64): Morton
    keys, or Peano-Hilbert keys with curve="hilbert"."""
    lib = lib or load()
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    n = pos.shape[0]
    lo, side = _box(lo, side)
    q = np.empty((n, 3), dtype=np.uint32)
    k = np.empty(n, dtype=np.uint64)
    if curve == "morton":
        rc = lib.tbo_keys(_ptr(pos), n, _ptr(lo), side, _ptr(q), _ptr(k))
    else:
        rc = lib.tbo_keys_curve(_ptr(pos), n, _ptr(lo), side, _curve(curve), _ptr(q), _ptr(k))
    if rc:
        raise OracleError(rc)
    return q, k


def hilbert_encode(q: np.ndarray, bits: int, lib=None) -> np.ndarray:
    """Index [N] (uint64, 3*bits bits, no leading 1) of cells q [N,3] on the
    Hilbert curve of `bits` levels."""
    lib = lib or load()
    q = np.ascontiguousarray(q, dtype=np.uint32).reshape(-1, 3)
    h = np.empty(q.shape[0], dtype=np.uint64)
    lib.tbo_hilbert_encode(_ptr(q), q.shape[0], int(bits), _ptr(h))
    return h


def hilbert_decode(h: np.ndarray, bits: int, lib=None) -> np.ndarray:
    """Cells [N,3] (uint32) of Hilbert indices h on the curve of `bits` levels."""
    lib = lib or load()
    h = np.ascontiguousarray(h, dtype=np.uint64).reshape(-1)
    q = np.empty((h.shape[0], 3), dtype=np.uint32)
    lib.tbo_hilbert_decode(_ptr(h), h.shape[0], int(bits), _ptr(q))
    return q


def max_cells(n: int, n_leaf: int, lib=None) -> int:
    lib = lib or load()
    return int(lib.tbo_max_cells(n, n_leaf))


ORACLE_STAGES = ("keys", "insertion", "perm", "canonical", "moments")
LEAF_FIRST_STAGES = ("keys", "sort", "reorder", "leaves", "parents", "output")


def build(pos: np.ndarray, mass: np.ndarray, n_leaf: int, lo=(0.0, 0.0, 0.0), side: float = 1.0,
          moments: bool = True, lib=None, curve: str = "morton") -> dict:
    """Reference tree.  Returns a dict of numpy arrays trimmed to n_cells:
    perm, dfs_perm, cell_key, cell_level, cell_first, cell_count, child_ptr [C,2],
    com [C,4] (dx, dy, dz relative to the cell centre, M), quad [C,6]
    (xx, xy, xz, yy, yz, zz), level_offset [23], n_cells, and stage_s: seconds
    of each step named in ORACLE_STAGES.  curve="hilbert": Peano-Hilbert keys."""
    lib = lib or load()
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, dtype=np.float32).reshape(-1)
    n = pos.shape[0]
    if mass.shape[0] != n:
        raise ValueError("pos and mass lengths differ")
    lo, side = _box(lo, side)
    cmax = max(max_cells(n, n_leaf, lib), 1)
    perm = np.empty(max(n, 1), dtype=np.int32)
    dfs = np.empty(max(n, 1), dtype=np.int32)
    key = np.empty(cmax, dtype=np.uint64)
    level = np.empty(cmax, dtype=np.uint8)
    first = np.empty(cmax, dtype=np.int32)
    count = np.empty(cmax, dtype=np.int32)
    child = np.empty((cmax, 2), dtype=np.int32)
    com = np.empty((cmax, 4), dtype=np.float64) if moments else None
    quad = np.empty((cmax, 6), dtype=np.float64) if moments else None
    loff = np.zeros(23, dtype=np.int64)
    nc = np.zeros(1, dtype=np.int64)
    stage = np.zeros(len(ORACLE_STAGES), dtype=np.float64)
    null = ctypes.c_void_p(0)
    outs = (_ptr(perm), _ptr(dfs), _ptr(key), _ptr(level), _ptr(first), _ptr(count), _ptr(child),
            _ptr(com) if moments else null, _ptr(quad) if moments else null, _ptr(loff), _ptr(nc),
            _ptr(stage))
    if curve == "morton":
        rc = lib.tbo_build_timed(_ptr(pos), _ptr(mass), n, n_leaf, _ptr(lo), side, *outs)
    else:
        rc = lib.tbo_build_curve(_ptr(pos), _ptr(mass), n, n_leaf, _ptr(lo), side,
                                 _curve(curve), *outs)
    if rc:
        raise OracleError(rc)
    c = int(nc[0])
    out = dict(perm=perm[:n], dfs_perm=dfs[:n], cell_key=key[:c], cell_level=level[:c],
               cell_first=first[:c], cell_count=count[:c], child_ptr=child[:c],
               level_offset=loff, n_cells=c, stage_s=dict(zip(ORACLE_STAGES, stage.tolist())))
    if moments:
        out["com"] = com[:c]
        out["quad"] = quad[:c]
    return out


def leaf_first_build(pos: np.ndarray, mass: np.ndarray, n_leaf: int, lo=(0.0, 0.0, 0.0),
                     side: float = 1.0, lib=None) -> dict:
    """The paper's leaf-first method on one CPU thread (tb_leaffirst.c), same
    output layout as build() (without dfs_perm); stage_s holds the seconds of
    each step named in LEAF_FIRST_STAGES."""
    lib = lib or load()
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, dtype=np.float32).reshape(-1)
    n = pos.shape[0]
    if mass.shape[0] != n:
        raise ValueError("pos and mass lengths differ")
    lo, side = _box(lo, side)
    cmax = max(max_cells(n, n_leaf, lib), 1)
    perm = np.empty(max(n, 1), dtype=np.int32)
    key = np.empty(cmax, dtype=np.uint64)
    level = np.empty(cmax, dtype=np.uint8)
    first = np.empty(cmax, dtype=np.int32)
    count = np.empty(cmax, dtype=np.int32)
    child = np.empty((cmax, 2), dtype=np.int32)
    com = np.empty((cmax, 4), dtype=np.float64)
    quad = np.empty((cmax, 6), dtype=np.float64)
    loff = np.zeros(23, dtype=np.int64)
    nc = np.zeros(1, dtype=np.int64)
    stage = np.zeros(len(LEAF_FIRST_STAGES), dtype=np.float64)
    rc = lib.tbl_build(_ptr(pos), _ptr(mass), n, n_leaf, _ptr(lo), side, _ptr(perm), _ptr(key),
                       _ptr(level), _ptr(first), _ptr(count), _ptr(child), _ptr(com), _ptr(quad),
                       _ptr(loff), _ptr(nc), _ptr(stage))
    if rc:
        raise OracleError(rc)
    c = int(nc[0])
    return dict(perm=perm[:n], cell_key=key[:c], cell_level=level[:c], cell_first=first[:c],
                cell_count=count[:c], child_ptr=child[:c], com=com[:c], quad=quad[:c],
                level_offset=loff, n_cells=c,
                stage_s=dict(zip(LEAF_FIRST_STAGES, stage.tolist())))


def cell_moments(pos, mass, perm, first: int, count: int, key: int, level: int,
                 lo=(0.0, 0.0, 0.0), side: float = 1.0, lib=None):
    """Moments of one cell from its particle range of ``perm`` (FP64, compensated)."""
    lib = lib or load()
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, dtype=np.float32).reshape(-1)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    lo, side = _box(lo, side)
    com = np.empty(4, dtype=np.float64)
    quad = np.empty(6, dtype=np.float64)
    rc = lib.tbo_cell_moments(_ptr(pos), _ptr(mass), _ptr(lo), side, _ptr(perm), int(first),
                              int(count), ctypes.c_uint64(int(key)), int(level), _ptr(com),
                              _ptr(quad))
    if rc:
        raise OracleError(rc)
    return com, quad


def direct_forces(pos, mass, eps: float = 0.0, lib=None) -> np.ndarray:
    """O(N^2) direct summation (Sec. 2.1), FP64: [N][4] = (ax, ay, az, phi) in input
    order, G = 1, Plummer softening eps, no self term."""
    lib = lib or load()
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, dtype=np.float32).reshape(-1)
    acc = np.zeros((pos.shape[0], 4), dtype=np.float64)
    rc = lib.tbg_direct(_ptr(pos), _ptr(mass), pos.shape[0], float(eps), _ptr(acc))
    if rc:
        raise OracleError(rc)
    return acc


def direct_forces_at(pos, mass, idx, eps: float = 0.0, lib=None) -> np.ndarray:
    """Direct summation for the particles idx only: [len(idx)][4] (ax, ay, az, phi)."""
    lib = lib or load()
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, dtype=np.float32).reshape(-1)
    idx = np.ascontiguousarray(idx, dtype=np.int64).reshape(-1)
    acc = np.zeros((idx.shape[0], 4), dtype=np.float64)
    rc = lib.tbg_direct_subset(_ptr(pos), _ptr(mass), pos.shape[0], float(eps), _ptr(idx),
                               idx.shape[0], _ptr(acc))
    if rc:
        raise OracleError(rc)
    return acc


def walk_forces(pos, mass, tree: dict, theta: float = 0.75, n_crit: int = 512, eps: float = 0.0,
                quadrupole: bool = True, lo=(0.0, 0.0, 0.0), side: float = 1.0, lib=None,
                curve: str = "morton"):
    """Sequential Barnes-Hut group walk over an oracle tree (build() output).
    Returns (acc [N][5] in sorted order: ax, ay, az, phi, sum of |terms|,
    stats dict with the number of groups and interactions)."""
    lib = lib or load()
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    mass = np.ascontiguousarray(mass, dtype=np.float32).reshape(-1)
    n = pos.shape[0]
    lo, side = _box(lo, side)
    acc = np.zeros((n, 5), dtype=np.float64)
    stats = np.zeros(2, dtype=np.int64)
    arrs = [np.ascontiguousarray(tree[k]) for k in ("perm", "cell_key", "cell_level", "cell_first",
                                                    "cell_count", "child_ptr", "com", "quad")]
    rc = lib.tbg_walk_tree_curve(_ptr(pos), _ptr(mass), _ptr(arrs[0]), n,
                                 *[_ptr(a) for a in arrs[1:]], _ptr(lo), side, float(theta),
                                 int(n_crit), float(eps), 1 if quadrupole else 0, _curve(curve),
                                 _ptr(acc), _ptr(stats))
    if rc:
        raise OracleError(rc)
    return acc, {"groups": int(stats[0]), "interactions": int(stats[1])}


def auto_box(pos, lib=None):
    """Root box chosen from the data: (lo[3], side)."""
    lib = lib or load()
    pos = np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3)
    lo = np.empty(3, dtype=np.float64)
    side = np.empty(1, dtype=np.float64)
    rc = lib.tbo_auto_box(_ptr(pos), pos.shape[0], _ptr(lo), _ptr(side))
    if rc:
        raise OracleError(rc)
    return lo, float(side[0])
