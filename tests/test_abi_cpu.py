"""The C-ABI library loads, exports every entry point its header declares, and
rejects bad arguments on the host before anything reaches a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2312_06102_amd import treebuild as tb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "treebuild.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(tb_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = tb.load_library()
    names = _declared()
    assert len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name
    assert set(tb.EXPORTS) <= set(names)


def test_header_constants_match_binding():
    text = open(HEADER).read()
    for name in ("TB_OK", "TB_ERR_ARG", "TB_ERR_BOX", "TB_ERR_WORKSPACE", "TB_ERR_HIP",
                 "TB_ERR_NONFINITE", "TB_ERR_MASS", "TB_ERR_INTERNAL", "TB_MAX_DEPTH", "TB_MAX_NLEAF"):
        m = re.search(rf"#define {name} \(?(-?\d+)\)?", text)
        assert m, name
        assert int(m.group(1)) == getattr(tb, name), name


def test_version():
    assert "gfx950" in tb.tb_version()


def test_max_cells():
    assert tb.tb_max_cells(0, 16) == 0
    assert tb.tb_max_cells(65536, 16) == 65536 + 21 * (65536 // 17)
    assert tb.tb_max_cells(1, 1) == 1
    for bad in [(-1, 16), (10, 0), (10, tb.TB_MAX_NLEAF + 1), (2 ** 31, 16)]:
        with pytest.raises(tb.TreeBuildArgError):
            tb.tb_max_cells(*bad)
    # C_max must fit the int32 child links
    with pytest.raises(tb.TreeBuildArgError):
        tb.tb_max_cells(2 ** 31 - 1, 1)


def test_workspace_bytes_grows_with_n():
    a = tb.tb_workspace_bytes(1000, 16)
    b = tb.tb_workspace_bytes(1 << 20, 16)
    assert 0 < a < b
    # keys x2, payload, look-back words: at least 20 B per particle
    assert b >= 20 * (1 << 20)
    assert tb.tb_workspace_bytes(0, 16) == 0
    with pytest.raises(tb.TreeBuildArgError):
        tb.tb_workspace_bytes(10, 16, flags=7)
    with pytest.raises(tb.TreeBuildArgError):
        tb.tb_workspace_bytes(10, 16, flags=tb.TB_SORT_CONFIG(200))
    # the look-back switch is a known flag; neighbouring bits are not.  Counted
    # passes keep one digit byte per element between passes, which look-back
    # passes (the default on a grid this small) do not need
    lb, dflt = tb.tb_workspace_bytes(10000, 16, tb.TB_SORT_LOOKBACK), tb.tb_workspace_bytes(10000, 16)
    cnt = tb.tb_workspace_bytes(10000, 16, tb.TB_SORT_COUNTED)
    assert dflt == lb
    assert abs((cnt - lb) - 10000) <= 256  # regions are 256-byte aligned
    # the subtree-rooted cell build is a known flag too
    assert tb.tb_workspace_bytes(10000, 16, tb.TB_SUBTREES) > 0
    assert tb.tb_workspace_bytes(10000, 16, tb.TB_SORT_COUNTED) > 0
    with pytest.raises(tb.TreeBuildArgError):
        tb.tb_workspace_bytes(10000, 16, tb.TB_SORT_COUNTED | tb.TB_SORT_LOOKBACK)
    assert tb.tb_workspace_bytes(10000, 16, tb.TB_HILBERT) > 0
    # the set-size bound of a batch is a known flag (bits 24..28)
    assert tb.tb_workspace_bytes_batched(10000, 8, 16, tb.TB_SET_INDEX_BITS(12)) > 0
    m = re.search(r"#define TB_SET_INDEX_BITS\(k\) \(\(\(\(uint32_t\)\(k\)\) & 0x1fu\) << 24\)",
                  open(HEADER).read())
    assert m and tb.TB_SET_INDEX_BITS(12) == 12 << 24
    for bit in (16, 21, 31):
        with pytest.raises(tb.TreeBuildArgError):
            tb.tb_workspace_bytes(10, 16, flags=1 << bit)


def test_lookback_flag_matches_header():
    m = re.search(r"#define TB_SORT_LOOKBACK \(1u << (\d+)\)", open(HEADER).read())
    assert m and (1 << int(m.group(1))) == tb.TB_SORT_LOOKBACK
    m = re.search(r"#define TB_SUBTREES \(1u << (\d+)\)", open(HEADER).read())
    assert m and (1 << int(m.group(1))) == tb.TB_SUBTREES
    m = re.search(r"#define TB_HILBERT \(1u << (\d+)\)", open(HEADER).read())
    assert m and (1 << int(m.group(1))) == tb.TB_HILBERT
    m = re.search(r"#define TB_SORT_COUNTED \(1u << (\d+)\)", open(HEADER).read())
    assert m and (1 << int(m.group(1))) == tb.TB_SORT_COUNTED


def test_sort_config_table():
    cfgs = tb.tb_sort_configs()
    assert cfgs[0] == (8, 11, 512)
    for k, (bits, ipt, threads) in enumerate(cfgs):
        assert 8 <= bits <= 9 and threads % 64 == 0
        assert tb.tb_workspace_bytes(4096, 16, tb.TB_SORT_CONFIG(k)) > 0


def _fake_tree():
    t = tb.TbTree()
    for i, (f, _) in enumerate(tb.TbTree._fields_):
        setattr(t, f, 0x1000 * (i + 1))
    t.box_out = t.pos_sorted = t.mass_sorted = t.key_sorted = None
    return t


def test_build_rejects_bad_arguments_before_launch():
    """Each of these returns synchronously; none of them touches device memory
    (the pointers are fake)."""
    t = _fake_tree()
    good_box = tb.TbBox()
    good_box.side = 1.0
    ws = 1 << 40
    call = lambda n, nl, box, flags, wsb, out: tb.tb_build(0x10, 0x20, n, nl, box, flags, 0x30, wsb,
                                                            out, 0)
    assert call(100, 0, good_box, 0, ws, t) == tb.TB_ERR_ARG
    assert call(-5, 16, good_box, 0, ws, t) == tb.TB_ERR_ARG
    assert call(100, 16, good_box, 99, ws, t) == tb.TB_ERR_ARG
    bad_box = tb.TbBox()
    bad_box.side = 3.0
    assert call(100, 16, bad_box, 0, ws, t) == tb.TB_ERR_BOX
    bad_box.side = 1.0
    bad_box.lo[1] = float("nan")
    assert call(100, 16, bad_box, 0, ws, t) == tb.TB_ERR_BOX
    bad_box.lo[1] = 0.0
    bad_box.side = -2.0
    assert call(100, 16, bad_box, 0, ws, t) == tb.TB_ERR_BOX
    assert call(100, 16, good_box, 0, 10, t) == tb.TB_ERR_WORKSPACE
    t2 = _fake_tree()
    t2.perm = None
    assert call(100, 16, good_box, 0, ws, t2) == tb.TB_ERR_ARG
    t3 = _fake_tree()
    t3.status = None
    assert call(0, 16, good_box, 0, ws, t3) == tb.TB_ERR_ARG


def test_trace_read_empty():
    tb.tb_trace_enable(False)
    assert tb.tb_trace_read() == {}


def test_binding_refuses_host_tensors():
    import torch
    pos = torch.zeros((10, 3), dtype=torch.float32)
    mass = torch.ones(10, dtype=torch.float32)
    with pytest.raises(ValueError, match="GPU"):
        tb._check_device_tensor(pos, "pos", torch.float32, (3,))
    with pytest.raises(Exception):
        tb.build(pos, mass, 16)


def test_no_oracle_in_product_path():
    """The product package never imports or links the oracle."""
    pkg = os.path.join(ROOT, "paper_2312_06102_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text and "tb_oracle" not in text, f


def test_batched_workspace_and_validation():
    one = tb.tb_workspace_bytes_batched(100000, 1, 16)
    assert one == tb.tb_workspace_bytes(100000, 16)
    many = tb.tb_workspace_bytes_batched(100000, 4096, 16)
    assert many > one
    assert tb.tb_workspace_bytes_batched(0, 7, 16) == 0
    for bad in [(100, 0, 16), (100, tb.TB_MAX_SETS + 1, 16), (100, 4, 0), (-1, 4, 16)]:
        with pytest.raises(tb.TreeBuildArgError):
            tb.tb_workspace_bytes_batched(*bad)
    t = _fake_tree()
    ws = 1 << 40
    call = lambda n, B, offs, nl=16, flags=0, wsb=ws: tb.tb_build_batched(
        0x10, 0x20, n, B, offs, nl, None, flags, 0x30, wsb, t, 0x40, 0)
    assert call(100, 0, 0x50) == tb.TB_ERR_ARG
    assert call(100, tb.TB_MAX_SETS + 1, 0x50) == tb.TB_ERR_ARG
    assert call(100, 4, None) == tb.TB_ERR_ARG
    assert call(100, 4, 0x50, nl=0) == tb.TB_ERR_ARG
    assert call(100, 4, 0x50, flags=77) == tb.TB_ERR_ARG
    assert call(100, 4, 0x50, wsb=16) == tb.TB_ERR_WORKSPACE


def test_status_bits_distinct():
    text = open(HEADER).read()
    bits = [int(re.search(rf"#define {n} (\d+)", text).group(1)) for n in
            ("TB_STATUS_NONFINITE", "TB_STATUS_MASS", "TB_STATUS_INTERNAL", "TB_STATUS_SETS",
             "TB_STATUS_BOX")]
    assert bits == [tb.TB_STATUS_NONFINITE, tb.TB_STATUS_MASS, tb.TB_STATUS_INTERNAL,
                    tb.TB_STATUS_SETS, tb.TB_STATUS_BOX]
    assert len(set(bits)) == 5 and all(b & (b - 1) == 0 for b in bits)
    assert int(re.search(r"#define TB_MAX_SETS (\d+)", text).group(1)) == tb.TB_MAX_SETS


def test_noalloc_rejects_oversize_on_the_host():
    """The build without allocation refuses a build whose workspace would not fit
    its fixed array before any HIP call (fake pointers, no GPU here), and checks
    its other arguments like tb_build."""
    t = _fake_tree()
    box = tb.TbBox()
    box.side = 1.0
    n = 1 << 24
    assert tb.tb_workspace_bytes(n, 16) > tb.TB_NOALLOC_SCRATCH_BYTES
    assert tb.tb_build_noalloc(0x10, 0x20, n, 16, box, 0, t, 0) == tb.TB_ERR_SCRATCH
    assert tb.tb_build_noalloc(0x10, 0x20, 100, 0, box, 0, t, 0) == tb.TB_ERR_ARG
    assert tb.tb_build_noalloc(0x10, 0x20, 100, 16, box, 99, t, 0) == tb.TB_ERR_ARG
    m = re.search(r"#define TB_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", open(HEADER).read())
    assert m and int(m.group(1)) << int(m.group(2)) == tb.TB_NOALLOC_SCRATCH_BYTES
