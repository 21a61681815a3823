"""Python binding of the gfx950 tree-build library (include/treebuild.h).

Argument marshalling only: every step of a build runs in the HIP kernels of
``libtreebuild.so``.  PyTorch supplies device memory and the stream.  There is
no CPU fallback: without the native library, or with tensors that are not on a
GPU, every call raises.

The functions ``tb_max_cells``, ``tb_workspace_bytes``,
``tb_workspace_bytes_batched``, ``tb_build``, ``tb_build_sync``, ``tb_build_noalloc``,
``tb_build_batched``, ``tb_build_batched_sync``, ``tb_trace_enable``,
``tb_trace_read``, ``tb_sort_configs`` and ``tb_version`` mirror the C entry
points of the same names.  ``Builder`` keeps a workspace and output buffers for
repeated builds of one set, ``BatchBuilder`` the same for batches of sets
stored back to back; ``build`` and ``build_batched`` are the one-shot forms.
Both builders can record their build into a HIP graph (``capture``) and replay
it (``replay``).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtreebuild.so")

TB_OK = 0
TB_ERR_ARG = -1
TB_ERR_BOX = -2
TB_ERR_WORKSPACE = -3
TB_ERR_HIP = -4
TB_ERR_NONFINITE = -5
TB_ERR_MASS = -6
TB_ERR_INTERNAL = -7
TB_ERR_SCRATCH = -8
TB_STATUS_NONFINITE = 1
TB_STATUS_MASS = 2
TB_STATUS_INTERNAL = 4
TB_STATUS_SETS = 8
TB_STATUS_BOX = 16
TB_FP64 = 0
TB_MIXED = 1
TB_SORT_LOOKBACK = 1 << 17  # keep the decoupled look-back in every radix pass
TB_SUBTREES = 1 << 18  # build the cells subtree by subtree (Sec. 2.3.3, eq. 2)
TB_SORT_COUNTED = 1 << 19  # count the tiles' digits in every radix pass
TB_HILBERT = 1 << 20  # Peano-Hilbert keys (footnote of Sec. 2.2)


def TB_SET_INDEX_BITS(k: int) -> int:
    """Batches: every set holds at most 2^k particles (the sort carries indices
    within the set in k bits)."""
    return (int(k) & 0x1F) << 24
CURVES = ("morton", "hilbert")


def _curve_flag(curve: str) -> int:
    if curve not in CURVES:
        raise ValueError(f"curve must be one of {CURVES}")
    return TB_HILBERT if curve == "hilbert" else 0
TB_MAX_DEPTH = 21
TB_MAX_NLEAF = 1024
TB_MAX_SETS = 16383
TB_NOALLOC_SCRATCH_BYTES = 64 << 20  # the fixed scratch array of tb_build_noalloc
TB_GRAV_QUADRUPOLE = 1

EXPORTS = ("tb_max_cells", "tb_workspace_bytes", "tb_workspace_bytes_batched", "tb_build",
           "tb_build_sync", "tb_build_noalloc", "tb_gravity_workspace_bytes", "tb_gravity",
           "tb_build_batched", "tb_build_batched_sync", "tb_kick_drift", "tb_permute",
           "tb_trace_enable",
           "tb_trace_read", "tb_sort_configs", "tb_version")

_ERRNAMES = {TB_ERR_ARG: "TB_ERR_ARG", TB_ERR_BOX: "TB_ERR_BOX", TB_ERR_WORKSPACE: "TB_ERR_WORKSPACE",
             TB_ERR_HIP: "TB_ERR_HIP", TB_ERR_NONFINITE: "TB_ERR_NONFINITE", TB_ERR_MASS: "TB_ERR_MASS",
             TB_ERR_INTERNAL: "TB_ERR_INTERNAL", TB_ERR_SCRATCH: "TB_ERR_SCRATCH"}


def TB_SORT_CONFIG(k: int) -> int:
    return (int(k) & 0xFF) << 8


class TbBox(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("side", ctypes.c_double)]


class TbTree(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in (
        "perm", "cell_key", "cell_level", "cell_first", "cell_count", "child_ptr", "com", "quad",
        "level_offset", "n_cells", "status", "box_out", "pos_sorted", "mass_sorted", "key_sorted")]


class TbTraceEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class TreeBuildError(RuntimeError):
    def __init__(self, code: int, what: str = "tb_build"):
        super().__init__(f"{what} failed: {_ERRNAMES.get(code, code)}")
        self.code = code


class TreeBuildArgError(TreeBuildError, ValueError):
    pass


def _raise(code: int, what: str):
    if code in (TB_ERR_ARG, TB_ERR_BOX, TB_ERR_WORKSPACE, TB_ERR_NONFINITE, TB_ERR_MASS,
                TB_ERR_SCRATCH):
        raise TreeBuildArgError(code, what)
    raise TreeBuildError(code, what)


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libtreebuild.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_2312_06102_amd.build_lib` (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.tb_max_cells.argtypes = [i64, i32, ctypes.POINTER(i64)]
    lib.tb_workspace_bytes.argtypes = [i64, i32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_size_t)]
    sig = [P, P, i64, i32, ctypes.POINTER(TbBox), ctypes.c_uint32, P, ctypes.c_size_t,
           ctypes.POINTER(TbTree), P]
    lib.tb_build.argtypes = sig
    lib.tb_build_sync.argtypes = sig
    lib.tb_build_noalloc.argtypes = [P, P, i64, i32, ctypes.POINTER(TbBox), ctypes.c_uint32,
                                     ctypes.POINTER(TbTree), P]
    lib.tb_gravity_workspace_bytes.argtypes = [i64, ctypes.POINTER(ctypes.c_size_t)]
    lib.tb_gravity.argtypes = [P, P, i64, ctypes.POINTER(TbTree), i64, ctypes.c_double, i32,
                               ctypes.c_double, ctypes.c_uint32, P, P, P, ctypes.c_size_t, P]
    lib.tb_workspace_bytes_batched.argtypes = [i64, i32, i32, ctypes.c_uint32,
                                               ctypes.POINTER(ctypes.c_size_t)]
    bsig = [P, P, i64, i32, P, i32, P, ctypes.c_uint32, P, ctypes.c_size_t,
            ctypes.POINTER(TbTree), P, P]
    lib.tb_build_batched.argtypes = bsig
    lib.tb_build_batched_sync.argtypes = bsig
    lib.tb_kick_drift.argtypes = [P, P, i64, ctypes.c_double, ctypes.c_double, P, P, P, P]
    lib.tb_permute.argtypes = [P, i64, P, i32, P, P, P]
    lib.tb_trace_enable.argtypes = [ctypes.c_int]
    lib.tb_trace_read.argtypes = [ctypes.POINTER(TbTraceEntry), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.tb_sort_configs.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.tb_version.restype = ctypes.c_char_p
    for f in EXPORTS[:-1]:
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


# ----------------------------------------------------------------------------
# the C entry points
# ----------------------------------------------------------------------------

def tb_max_cells(n: int, n_leaf: int) -> int:
    out = ctypes.c_int64(0)
    rc = load_library().tb_max_cells(int(n), int(n_leaf), ctypes.byref(out))
    if rc:
        _raise(rc, "tb_max_cells")
    return out.value


def tb_workspace_bytes(n: int, n_leaf: int, flags: int = TB_FP64) -> int:
    out = ctypes.c_size_t(0)
    rc = load_library().tb_workspace_bytes(int(n), int(n_leaf), int(flags), ctypes.byref(out))
    if rc:
        _raise(rc, "tb_workspace_bytes")
    return out.value


def tb_build(pos_ptr: int, mass_ptr: int, n: int, n_leaf: int, box: Optional[TbBox], flags: int,
             ws_ptr: int, ws_bytes: int, out: TbTree, stream: int) -> int:
    """Raw call: device pointers as ints; returns the C return code."""
    return load_library().tb_build(ctypes.c_void_p(pos_ptr), ctypes.c_void_p(mass_ptr), int(n),
                                   int(n_leaf), ctypes.byref(box) if box is not None else None,
                                   int(flags), ctypes.c_void_p(ws_ptr), int(ws_bytes),
                                   ctypes.byref(out), ctypes.c_void_p(stream))


def tb_build_sync(pos_ptr: int, mass_ptr: int, n: int, n_leaf: int, box: Optional[TbBox],
                  flags: int, ws_ptr: int, ws_bytes: int, out: TbTree, stream: int) -> int:
    return load_library().tb_build_sync(ctypes.c_void_p(pos_ptr), ctypes.c_void_p(mass_ptr), int(n),
                                        int(n_leaf), ctypes.byref(box) if box is not None else None,
                                        int(flags), ctypes.c_void_p(ws_ptr), int(ws_bytes),
                                        ctypes.byref(out), ctypes.c_void_p(stream))


def tb_build_noalloc(pos_ptr: int, mass_ptr: int, n: int, n_leaf: int, box: Optional[TbBox],
                     flags: int, out: TbTree, stream: int) -> int:
    """Raw call of the build that allocates nothing (scratch in the library's fixed
    device array); returns the C return code."""
    return load_library().tb_build_noalloc(ctypes.c_void_p(pos_ptr), ctypes.c_void_p(mass_ptr),
                                           int(n), int(n_leaf),
                                           ctypes.byref(box) if box is not None else None,
                                           int(flags), ctypes.byref(out), ctypes.c_void_p(stream))


def tb_gravity_workspace_bytes(c_max: int) -> int:
    out = ctypes.c_size_t(0)
    rc = load_library().tb_gravity_workspace_bytes(int(c_max), ctypes.byref(out))
    if rc:
        _raise(rc, "tb_gravity_workspace_bytes")
    return out.value


def tb_gravity(pos_ptr: int, mass_ptr: int, n: int, tree: TbTree, c_max: int, theta: float,
               n_crit: int, eps: float, flags: int, acc_ptr: int, stats_ptr: Optional[int],
               ws_ptr: int, ws_bytes: int, stream: int) -> int:
    """Raw call of the tree walk: device pointers as ints; returns the C code."""
    return load_library().tb_gravity(ctypes.c_void_p(pos_ptr), ctypes.c_void_p(mass_ptr), int(n),
                                     ctypes.byref(tree), int(c_max), float(theta), int(n_crit),
                                     float(eps), int(flags), ctypes.c_void_p(acc_ptr),
                                     ctypes.c_void_p(stats_ptr), ctypes.c_void_p(ws_ptr),
                                     int(ws_bytes), ctypes.c_void_p(stream))


def tb_kick_drift(perm_ptr: Optional[int], acc_ptr: int, n: int, dt_kick: float, dt_drift: float,
                  pos_ptr: int, vel_ptr: int, status_ptr: Optional[int], stream: int) -> int:
    """Raw call of the leapfrog update: device pointers as ints; returns the C code."""
    return load_library().tb_kick_drift(ctypes.c_void_p(perm_ptr), ctypes.c_void_p(acc_ptr),
                                        int(n), float(dt_kick), float(dt_drift),
                                        ctypes.c_void_p(pos_ptr), ctypes.c_void_p(vel_ptr),
                                        ctypes.c_void_p(status_ptr), ctypes.c_void_p(stream))


def tb_permute(perm_ptr: int, n: int, src_ptr: int, width: int, dst_ptr: int,
               status_ptr: Optional[int], stream: int) -> int:
    """Raw call of the row gather dst[s] = src[perm[s]]; returns the C code."""
    return load_library().tb_permute(ctypes.c_void_p(perm_ptr), int(n), ctypes.c_void_p(src_ptr),
                                     int(width), ctypes.c_void_p(dst_ptr),
                                     ctypes.c_void_p(status_ptr), ctypes.c_void_p(stream))


def kick_drift(perm: Optional[torch.Tensor], acc: torch.Tensor, dt_kick: float, dt_drift: float,
               pos: torch.Tensor, vel: torch.Tensor, status: Optional[torch.Tensor] = None,
               stream=None) -> None:
    """vel[perm[s]] += acc[s] dt_kick; pos[perm[s]] += vel[perm[s]] dt_drift (in place)."""
    n = pos.shape[0]
    _check_device_tensor(pos, "pos", torch.float32, (3,))
    _check_device_tensor(vel, "vel", torch.float32, (3,))
    _check_device_tensor(acc, "acc", torch.float64, (4,))
    if vel.shape[0] != n or acc.shape[0] < n or (perm is not None and perm.shape[0] < n):
        raise ValueError("pos, vel, acc and perm must describe the same particles")
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = tb_kick_drift(perm.data_ptr() if perm is not None else None, acc.data_ptr(), n, dt_kick,
                       dt_drift, pos.data_ptr(), vel.data_ptr(),
                       status.data_ptr() if status is not None else None, s.cuda_stream)
    if rc:
        _raise(rc, "tb_kick_drift")


def permute(perm: torch.Tensor, src: torch.Tensor, dst: torch.Tensor,
            status: Optional[torch.Tensor] = None, stream=None) -> None:
    """dst[s] = src[perm[s]] for rows of 4-byte elements (float32 or int32)."""
    n = perm.shape[0]
    if src.dtype not in (torch.float32, torch.int32) or dst.dtype != src.dtype:
        raise ValueError("permute moves float32 or int32 rows")
    if not (src.is_cuda and dst.is_cuda and perm.is_cuda and src.is_contiguous()
            and dst.is_contiguous()):
        raise ValueError("permute needs contiguous device tensors")
    width = 1 if src.dim() == 1 else int(src[0].numel())
    if src.shape != dst.shape or src.shape[0] != n:
        raise ValueError("src and dst must be [N] or [N][width] with N = len(perm)")
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = tb_permute(perm.data_ptr(), n, src.data_ptr(), width, dst.data_ptr(),
                    status.data_ptr() if status is not None else None, s.cuda_stream)
    if rc:
        _raise(rc, "tb_permute")


def tb_workspace_bytes_batched(n_total: int, nsets: int, n_leaf: int, flags: int = TB_FP64) -> int:
    out = ctypes.c_size_t(0)
    rc = load_library().tb_workspace_bytes_batched(int(n_total), int(nsets), int(n_leaf), int(flags),
                                                   ctypes.byref(out))
    if rc:
        _raise(rc, "tb_workspace_bytes_batched")
    return out.value


def tb_build_batched(pos_ptr: int, mass_ptr: int, n_total: int, nsets: int, offsets_ptr: int,
                     n_leaf: int, boxes_ptr: Optional[int], flags: int, ws_ptr: int, ws_bytes: int,
                     out: TbTree, cell_offsets_ptr: Optional[int], stream: int) -> int:
    """Raw call: device pointers as ints (boxes / cell_offsets may be None)."""
    return load_library().tb_build_batched(
        ctypes.c_void_p(pos_ptr), ctypes.c_void_p(mass_ptr), int(n_total), int(nsets),
        ctypes.c_void_p(offsets_ptr), int(n_leaf), ctypes.c_void_p(boxes_ptr), int(flags),
        ctypes.c_void_p(ws_ptr), int(ws_bytes), ctypes.byref(out),
        ctypes.c_void_p(cell_offsets_ptr), ctypes.c_void_p(stream))


def tb_build_batched_sync(pos_ptr: int, mass_ptr: int, n_total: int, nsets: int, offsets_ptr: int,
                          n_leaf: int, boxes_ptr: Optional[int], flags: int, ws_ptr: int,
                          ws_bytes: int, out: TbTree, cell_offsets_ptr: Optional[int],
                          stream: int) -> int:
    return load_library().tb_build_batched_sync(
        ctypes.c_void_p(pos_ptr), ctypes.c_void_p(mass_ptr), int(n_total), int(nsets),
        ctypes.c_void_p(offsets_ptr), int(n_leaf), ctypes.c_void_p(boxes_ptr), int(flags),
        ctypes.c_void_p(ws_ptr), int(ws_bytes), ctypes.byref(out),
        ctypes.c_void_p(cell_offsets_ptr), ctypes.c_void_p(stream))


def tb_trace_enable(on: bool = True) -> None:
    load_library().tb_trace_enable(1 if on else 0)


def tb_trace_read() -> dict:
    """{kernel name: (launches, total_ms)}; resets the accumulators."""
    lib = load_library()
    cap = 64
    arr = (TbTraceEntry * cap)()
    cnt = ctypes.c_int(0)
    rc = lib.tb_trace_read(arr, cap, ctypes.byref(cnt))
    if rc:
        _raise(rc, "tb_trace_read")
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(cnt.value)}


def tb_sort_configs() -> list:
    """[(digit bits, keys per thread, threads)] indexed by TB_SORT_CONFIG(k)."""
    lib = load_library()
    cnt = ctypes.c_int(0)
    lib.tb_sort_configs(None, 0, ctypes.byref(cnt))
    arr = (ctypes.c_int32 * (3 * cnt.value))()
    lib.tb_sort_configs(arr, cnt.value, ctypes.byref(cnt))
    return [tuple(arr[3 * k:3 * k + 3]) for k in range(cnt.value)]


def tb_version() -> str:
    return load_library().tb_version().decode()


# ----------------------------------------------------------------------------
# torch-side buffers
# ----------------------------------------------------------------------------

def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _check_device_tensor(t: torch.Tensor, name: str, dtype, shape_tail=()):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU (no CPU path exists)")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} has shape {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


@dataclass
class TreeBuffers:
    """Device output buffers of one build (sized for C_max cells)."""
    perm: torch.Tensor
    cell_key: torch.Tensor
    cell_level: torch.Tensor
    cell_first: torch.Tensor
    cell_count: torch.Tensor
    child_ptr: torch.Tensor
    com: torch.Tensor
    quad: torch.Tensor
    level_offset: torch.Tensor
    n_cells: torch.Tensor
    status: torch.Tensor
    box_out: torch.Tensor
    pos_sorted: Optional[torch.Tensor] = None
    mass_sorted: Optional[torch.Tensor] = None
    key_sorted: Optional[torch.Tensor] = None

    @staticmethod
    def allocate(n: int, n_leaf: int, precision: str = "fp64", device="cuda",
                 sorted_particles: bool = False, sorted_keys: bool = False,
                 nsets: int = 1) -> "TreeBuffers":
        cmax = max(tb_max_cells(n, n_leaf), 1)
        fdt = torch.float64 if precision == "fp64" else torch.float32
        kw = dict(device=device)
        nn = max(n, 1)
        return TreeBuffers(
            perm=torch.empty(nn, dtype=torch.int32, **kw),
            cell_key=torch.empty(cmax, dtype=torch.int64, **kw),  # uint64 bit patterns
            cell_level=torch.empty(cmax, dtype=torch.uint8, **kw),
            cell_first=torch.empty(cmax, dtype=torch.int32, **kw),
            cell_count=torch.empty(cmax, dtype=torch.int32, **kw),
            child_ptr=torch.empty((cmax, 2), dtype=torch.int32, **kw),
            com=torch.empty((cmax, 4), dtype=fdt, **kw),
            quad=torch.empty((cmax, 6), dtype=fdt, **kw),
            level_offset=torch.empty(TB_MAX_DEPTH + 2, dtype=torch.int64, **kw) if nsets == 1
            else torch.empty((nsets, TB_MAX_DEPTH + 2), dtype=torch.int64, **kw),
            n_cells=torch.empty(1, dtype=torch.int64, **kw),
            status=torch.empty(1, dtype=torch.int32, **kw),
            box_out=torch.empty(4, dtype=torch.float64, **kw) if nsets == 1
            else torch.empty((nsets, 4), dtype=torch.float64, **kw),
            pos_sorted=torch.empty((nn, 3), dtype=torch.float32, **kw) if sorted_particles else None,
            mass_sorted=torch.empty(nn, dtype=torch.float32, **kw) if sorted_particles else None,
            key_sorted=torch.empty(nn, dtype=torch.int64, **kw) if sorted_keys else None,
        )

    def struct(self) -> TbTree:
        t = TbTree()
        for f, _ in TbTree._fields_:
            v = getattr(self, f)
            setattr(t, f, _ptr(v))
        return t


def _box_struct(box) -> Optional[TbBox]:
    if box is None:
        return None
    lo, side = box
    b = TbBox()
    for a in range(3):
        b.lo[a] = float(lo[a])
    b.side = float(side)
    return b


def _check_status(st: int, what: str) -> None:
    if st & TB_STATUS_NONFINITE:
        _raise(TB_ERR_NONFINITE, what)
    if st & TB_STATUS_MASS:
        _raise(TB_ERR_MASS, what)
    if st & TB_STATUS_SETS:
        _raise(TB_ERR_ARG, what)
    if st & TB_STATUS_BOX:
        _raise(TB_ERR_BOX, what)
    if st & TB_STATUS_INTERNAL:
        _raise(TB_ERR_INTERNAL, what)


class _Graphable:
    """Records one launch() into a HIP graph (through torch's graph capture on a
    side stream) and replays it.  A build holds no memset node and no host
    synchronisation, so the captured graph is the plain kernel sequence."""

    _graph = None

    def capture(self, *args, **kwargs) -> None:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.launch(*args, **kwargs)  # resolves kernel attributes outside the capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.launch(*args, **kwargs)
        self._graph = g

    def replay(self) -> None:
        if self._graph is None:
            raise RuntimeError("capture() first")
        self._graph.replay()


class Builder(_Graphable):
    """Reusable workspace + outputs for repeated builds of N particles."""

    def __init__(self, n: int, n_leaf: int = 16, precision: str = "fp64", sort_config: int = 0,
                 device="cuda", sorted_particles: bool = False, sorted_keys: bool = False,
                 lookback: bool = False, subtrees: bool = False, counted: bool = False,
                 curve: str = "morton"):
        if precision not in ("fp64", "mixed"):
            raise ValueError("precision must be 'fp64' or 'mixed'")
        self.n, self.n_leaf, self.precision = int(n), int(n_leaf), precision
        self.flags = ((TB_FP64 if precision == "fp64" else TB_MIXED) | TB_SORT_CONFIG(sort_config)
                      | (TB_SORT_LOOKBACK if lookback else 0) | (TB_SUBTREES if subtrees else 0)
                      | (TB_SORT_COUNTED if counted else 0) | _curve_flag(curve))
        self.ws_bytes = tb_workspace_bytes(self.n, self.n_leaf, self.flags)
        self.workspace = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device)
        self.out = TreeBuffers.allocate(self.n, self.n_leaf, precision, device, sorted_particles,
                                        sorted_keys)
        self._struct = self.out.struct()

    def launch(self, pos: torch.Tensor, mass: torch.Tensor, box=None, stream=None) -> None:
        """Asynchronous build on `stream` (default: torch's current stream)."""
        _check_device_tensor(pos, "pos", torch.float32, (3,))
        _check_device_tensor(mass, "mass", torch.float32)
        if pos.shape[0] != self.n or mass.shape[0] != self.n:
            raise ValueError(f"this Builder is sized for N={self.n}")
        s = stream if stream is not None else torch.cuda.current_stream()
        rc = tb_build(pos.data_ptr(), mass.data_ptr(), self.n, self.n_leaf, _box_struct(box),
                      self.flags, self.workspace.data_ptr(), self.ws_bytes, self._struct,
                      s.cuda_stream)
        if rc:
            _raise(rc, "tb_build")

    def result(self) -> dict:
        """Synchronise and return the outputs trimmed to n_cells (device tensors)."""
        torch.cuda.synchronize()
        _check_status(int(self.out.status.item()), "tb_build")
        c = int(self.out.n_cells.item())
        o = self.out
        res = dict(perm=o.perm[:self.n], cell_key=o.cell_key[:c], cell_level=o.cell_level[:c],
                   cell_first=o.cell_first[:c], cell_count=o.cell_count[:c],
                   child_ptr=o.child_ptr[:c], com=o.com[:c], quad=o.quad[:c],
                   level_offset=o.level_offset.clone(), n_cells=c, box=o.box_out.clone())
        if o.pos_sorted is not None:
            res["pos_sorted"] = o.pos_sorted[:self.n]
            res["mass_sorted"] = o.mass_sorted[:self.n]
        if o.key_sorted is not None:
            res["key_sorted"] = o.key_sorted[:self.n]
        return res


    def gravity(self, theta: float = 0.75, n_crit: int = 512, eps: float = 0.0,
                quadrupole: bool = True, stream=None):
        """Barnes-Hut accelerations and potentials (tb_gravity) from the last
        build, which must be FP64 with sorted_particles=True.  Returns
        (acc [N][4] float64 device tensor in key order: ax, ay, az, phi;
        stats dict with the number of groups and of interactions)."""
        if self.precision != "fp64" or self.out.pos_sorted is None:
            raise ValueError("gravity needs an FP64 Builder with sorted_particles=True")
        c_max = max(tb_max_cells(self.n, self.n_leaf), 1)
        if getattr(self, "_grav_ws", None) is None:
            self._grav_ws_bytes = tb_gravity_workspace_bytes(c_max)
            self._grav_ws = torch.empty(self._grav_ws_bytes, dtype=torch.uint8,
                                        device=self.workspace.device)
        acc = torch.empty((max(self.n, 1), 4), dtype=torch.float64, device=self.workspace.device)
        stats = torch.zeros(2, dtype=torch.int64, device=self.workspace.device)
        s = stream if stream is not None else torch.cuda.current_stream()
        rc = tb_gravity(self.out.pos_sorted.data_ptr(), self.out.mass_sorted.data_ptr(), self.n,
                        self._struct, c_max, theta, n_crit, eps,
                        (TB_GRAV_QUADRUPOLE if quadrupole else 0) | (self.flags & TB_HILBERT),
                        acc.data_ptr(),
                        stats.data_ptr(), self._grav_ws.data_ptr(), self._grav_ws_bytes,
                        s.cuda_stream)
        if rc:
            _raise(rc, "tb_gravity")
        torch.cuda.synchronize()
        _check_status(int(self.out.status.item()), "tb_gravity")
        st = stats.cpu().tolist()
        return acc[:self.n], {"groups": st[0], "interactions": st[1]}


def build(pos: torch.Tensor, mass: torch.Tensor, n_leaf: int = 16, box=None,
          precision: str = "fp64", sort_config: int = 0, sorted_particles: bool = False,
          sorted_keys: bool = False, lookback: bool = False, subtrees: bool = False,
          counted: bool = False, curve: str = "morton") -> dict:
    """One-shot build; returns device tensors trimmed to n_cells.

    box: None (derive from data) or (lo[3], side) with side a power of two.
    lookback: keep the decoupled look-back in every radix pass (TB_SORT_LOOKBACK).
    subtrees: build the cells block by block from subtree roots (TB_SUBTREES); the
    tree is the same.
    counted: count the tiles' digits in every radix pass (TB_SORT_COUNTED).
    curve: "morton" or "hilbert" (TB_HILBERT: Peano-Hilbert keys).
    cell_key is returned as int64 holding the uint64 bit pattern."""
    b = Builder(pos.shape[0], n_leaf, precision, sort_config, pos.device, sorted_particles,
                sorted_keys, lookback, subtrees, counted, curve)
    b.launch(pos, mass, box)
    return b.result()


class BatchBuilder(_Graphable):
    """Reusable workspace + outputs for batches of `nsets` sets holding `n_total`
    particles together, stored back to back (set b = particles
    [set_offsets[b], set_offsets[b+1]))."""

    def __init__(self, n_total: int, nsets: int, n_leaf: int = 16, precision: str = "fp64",
                 sort_config: int = 0, device="cuda", sorted_particles: bool = False,
                 sorted_keys: bool = False, lookback: bool = False, subtrees: bool = False,
                 counted: bool = False, curve: str = "morton", set_index_bits: int = 0):
        """set_index_bits: k > 0 promises that every set holds at most 2^k
        particles (TB_SET_INDEX_BITS); a larger set is reported as
        TB_STATUS_SETS."""
        if precision not in ("fp64", "mixed"):
            raise ValueError("precision must be 'fp64' or 'mixed'")
        if not 0 <= int(set_index_bits) <= 31:
            raise ValueError("set_index_bits must be 0 (no bound) or 1 .. 31")
        self.n, self.nsets, self.n_leaf, self.precision = int(n_total), int(nsets), int(n_leaf), precision
        self.flags = ((TB_FP64 if precision == "fp64" else TB_MIXED) | TB_SORT_CONFIG(sort_config)
                      | (TB_SORT_LOOKBACK if lookback else 0) | (TB_SUBTREES if subtrees else 0)
                      | (TB_SORT_COUNTED if counted else 0) | _curve_flag(curve)
                      | TB_SET_INDEX_BITS(set_index_bits))
        self.ws_bytes = tb_workspace_bytes_batched(self.n, self.nsets, self.n_leaf, self.flags)
        self.workspace = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device)
        self.out = TreeBuffers.allocate(self.n, self.n_leaf, precision, device, sorted_particles,
                                        sorted_keys, nsets=self.nsets)
        if self.nsets == 1:  # keep the [B][23] / [B][4] shapes for one set too
            self.out.level_offset = self.out.level_offset.view(1, -1)
            self.out.box_out = self.out.box_out.view(1, -1)
        self.cell_offsets = torch.empty(self.nsets + 1, dtype=torch.int64, device=device)
        self._struct = self.out.struct()

    def launch(self, pos: torch.Tensor, mass: torch.Tensor, set_offsets: torch.Tensor,
               boxes: Optional[torch.Tensor] = None, stream=None) -> None:
        """Asynchronous batched build.  set_offsets: int64 [B+1] on the GPU;
        boxes: float64 [B][4] (lo, side) on the GPU, or None (boxes from data)."""
        _check_device_tensor(pos, "pos", torch.float32, (3,))
        _check_device_tensor(mass, "mass", torch.float32)
        _check_device_tensor(set_offsets, "set_offsets", torch.int64)
        if pos.shape[0] != self.n or mass.shape[0] != self.n:
            raise ValueError(f"this BatchBuilder is sized for n_total={self.n}")
        if set_offsets.shape[0] != self.nsets + 1:
            raise ValueError(f"set_offsets must hold nsets + 1 = {self.nsets + 1} entries")
        if boxes is not None:
            _check_device_tensor(boxes, "boxes", torch.float64, (4,))
            if boxes.shape[0] != self.nsets:
                raise ValueError("boxes must be [nsets][4]")
        s = stream if stream is not None else torch.cuda.current_stream()
        rc = tb_build_batched(pos.data_ptr(), mass.data_ptr(), self.n, self.nsets,
                              set_offsets.data_ptr(), self.n_leaf, _ptr(boxes), self.flags,
                              self.workspace.data_ptr(), self.ws_bytes, self._struct,
                              self.cell_offsets.data_ptr(), s.cuda_stream)
        if rc:
            _raise(rc, "tb_build_batched")

    def result(self) -> dict:
        """Synchronise and return the outputs trimmed to n_cells (device tensors)."""
        torch.cuda.synchronize()
        _check_status(int(self.out.status.item()), "tb_build_batched")
        c = int(self.out.n_cells.item())
        o = self.out
        res = dict(perm=o.perm[:self.n], cell_key=o.cell_key[:c], cell_level=o.cell_level[:c],
                   cell_first=o.cell_first[:c], cell_count=o.cell_count[:c],
                   child_ptr=o.child_ptr[:c], com=o.com[:c], quad=o.quad[:c],
                   level_offset=o.level_offset.clone(), n_cells=c, box=o.box_out.clone(),
                   cell_offsets=self.cell_offsets.clone())
        if o.pos_sorted is not None:
            res["pos_sorted"] = o.pos_sorted[:self.n]
            res["mass_sorted"] = o.mass_sorted[:self.n]
        if o.key_sorted is not None:
            res["key_sorted"] = o.key_sorted[:self.n]
        return res


def build_batched(pos: torch.Tensor, mass: torch.Tensor, set_offsets: torch.Tensor,
                  n_leaf: int = 16, boxes: Optional[torch.Tensor] = None,
                  precision: str = "fp64", sort_config: int = 0, sorted_particles: bool = False,
                  sorted_keys: bool = False, lookback: bool = False,
                  subtrees: bool = False, counted: bool = False, curve: str = "morton",
                  set_index_bits: int = 0) -> dict:
    """One-shot batched build; returns device tensors trimmed to n_cells."""
    b = BatchBuilder(pos.shape[0], set_offsets.shape[0] - 1, n_leaf, precision, sort_config,
                     pos.device, sorted_particles, sorted_keys, lookback, subtrees, counted,
                     curve, set_index_bits)
    b.launch(pos, mass, set_offsets, boxes)
    return b.result()
