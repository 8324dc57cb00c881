"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every entry point declared in include/abx.h,
and reject bad arguments before touching the device.
"""
import ctypes as C
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "abx.h")


def _lib():
    from paper_1908_11807_amd import abx
    if not os.path.exists(abx.LIB_PATH):
        from paper_1908_11807_amd import build
        build.build_library(verbose=False)
    return abx, abx.library()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(abx_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("abx_bvh_build", "abx_query_spatial", "abx_query_nearest"):
        assert required in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol():
    abx, L = _lib()
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing


def test_exported_symbols_match_nm():
    import subprocess
    abx, _ = _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", abx.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (abx_[a-z0-9_]+)\b", out))
    assert set(declared_symbols()) <= exported


def test_status_strings_and_version():
    abx, L = _lib()
    for s in range(9):
        assert L.abx_status_string(s)
    assert b"unknown" not in L.abx_status_string(8)
    assert "gfx950" in abx.version()


def test_build_sizes_validation():
    abx, L = _lib()
    tb, sb = C.c_size_t(), C.c_size_t()
    opt = abx.BuildOptions(abx.NODES_FP32, 21)
    bad_kind = abx.Primitives(7, None, 10)
    assert L.abx_bvh_build_sizes(C.byref(bad_kind), C.byref(opt), C.byref(tb), C.byref(sb)) == abx.ERR_INVALID_ARG
    neg = abx.Primitives(abx.PRIM_POINTS, None, -1)
    assert L.abx_bvh_build_sizes(C.byref(neg), C.byref(opt), C.byref(tb), C.byref(sb)) == abx.ERR_INVALID_ARG
    big = abx.Primitives(abx.PRIM_POINTS, 1, 2 ** 31)
    assert L.abx_bvh_build_sizes(C.byref(big), C.byref(opt), C.byref(tb), C.byref(sb)) == abx.ERR_OVERFLOW
    nulldata = abx.Primitives(abx.PRIM_POINTS, None, 5)
    assert L.abx_bvh_build_sizes(C.byref(nulldata), C.byref(opt), C.byref(tb), C.byref(sb)) == abx.ERR_INVALID_ARG
    bits = abx.BuildOptions(abx.NODES_FP32, 16)
    ok = abx.Primitives(abx.PRIM_POINTS, 1, 5)
    assert L.abx_bvh_build_sizes(C.byref(ok), C.byref(bits), C.byref(tb), C.byref(sb)) == abx.ERR_INVALID_ARG
    fmt = abx.BuildOptions(5, 21)
    assert L.abx_bvh_build_sizes(C.byref(ok), C.byref(fmt), C.byref(tb), C.byref(sb)) == abx.ERR_INVALID_ARG


@pytest.mark.parametrize("fmt,kind,lb", [(0, 0, 4), (0, 1, 4), (1, 0, 4), (1, 1, 32)])
def test_build_sizes_layout(fmt, kind, lb):
    abx, L = _lib()
    n = 1000
    tb, sb = C.c_size_t(), C.c_size_t()
    pr = abx.Primitives(kind, 1, n)
    opt = abx.BuildOptions(fmt, 21)
    assert L.abx_bvh_build_sizes(C.byref(pr), C.byref(opt), C.byref(tb), C.byref(sb)) == abx.OK
    nb = 64 if fmt == 0 else 32
    expect = 256 + -(-(n - 1) * nb // 256) * 256 + -(-n * lb // 256) * 256
    assert tb.value == expect
    assert sb.value > 0


def test_build_rejects_null_buffers_without_gpu():
    abx, L = _lib()
    pr = abx.Primitives(abx.PRIM_POINTS, 1, 10)
    opt = abx.BuildOptions(0, 21)
    h = C.c_void_p()
    assert L.abx_bvh_build(C.byref(pr), C.byref(opt), None, 0, None, 0, None, C.byref(h)) == abx.ERR_INVALID_ARG


def test_query_entry_points_reject_null_handle():
    abx, L = _lib()
    sb = C.c_size_t()
    pr = abx.Predicates(0, 1, 10, None, 1.0, 1)
    assert L.abx_query_spatial_sizes(None, C.byref(pr), C.byref(sb)) == abx.ERR_INVALID_ARG
    assert L.abx_query_nearest_sizes(None, 10, 3, C.byref(sb)) == abx.ERR_INVALID_ARG
    t = C.c_int64()
    assert L.abx_query_spatial(None, C.byref(pr), None, 0, None, None, 0, C.byref(t), None) == abx.ERR_INVALID_ARG
    assert L.abx_query_nearest(None, None, 10, 3, 1, None, 0, None, None, None, None) == abx.ERR_INVALID_ARG


def test_sort_and_morton_validation():
    abx, L = _lib()
    sb = C.c_size_t()
    assert L.abx_radix_sort_sizes(10, 0, C.byref(sb)) == abx.ERR_INVALID_ARG
    assert L.abx_radix_sort_sizes(10, 65, C.byref(sb)) == abx.ERR_INVALID_ARG
    assert L.abx_radix_sort_sizes(1000, 30, C.byref(sb)) == abx.OK and sb.value > 0
    assert L.abx_morton_codes(0, None, 10, None, 21, None, None) == abx.ERR_INVALID_ARG
    assert L.abx_morton_codes(0, 1, 10, 1, 15, 1, None) == abx.ERR_INVALID_ARG


def test_timing_registry_without_launches():
    abx, L = _lib()
    abx.timing_reset()
    assert abx.timing_get("nearest") == (0.0, 0)


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1908_11807_amd import abx
    monkeypatch.setattr(abx, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(abx, "_LIB", None)
    with pytest.raises(RuntimeError, match="not built"):
        abx.library()


def test_forest_sizes_validation():
    import numpy as np
    abx, L = _lib()
    off = np.array([0, 10, 10, 25], np.int64)
    pr = abx.ForestPrimitives(3, off.ctypes.data, 1, 1, 0)
    tb, sb = C.c_size_t(), C.c_size_t()
    assert L.abx_forest_build_sizes(C.byref(pr), C.byref(tb), C.byref(sb)) == abx.OK
    assert tb.value > 256 and sb.value > 0
    bad = np.array([0, 10, 5, 25], np.int64)              # decreasing offsets
    pr = abx.ForestPrimitives(3, bad.ctypes.data, 1, 1, 0)
    assert L.abx_forest_build_sizes(C.byref(pr), C.byref(tb), C.byref(sb)) == abx.ERR_INVALID_ARG
    pr = abx.ForestPrimitives(0, off.ctypes.data, 1, 1, 0)   # no trees
    assert L.abx_forest_build_sizes(C.byref(pr), C.byref(tb), C.byref(sb)) == abx.ERR_INVALID_ARG
    pr = abx.ForestPrimitives(513, off.ctypes.data, 1, 1, 0)  # too many trees
    assert L.abx_forest_build_sizes(C.byref(pr), C.byref(tb), C.byref(sb)) == abx.ERR_INVALID_ARG
    assert L.abx_graph_begin(None) == abx.ERR_INVALID_ARG     # null stream cannot be captured


def test_onepass_validation_without_gpu():
    abx, L = _lib()
    sb = C.c_size_t()
    pr = abx.Predicates(0, 1, 10, None, 1.0, 1)
    assert L.abx_query_spatial_1p_sizes(None, C.byref(pr), 4, C.byref(sb)) == abx.ERR_INVALID_ARG
    info = C.c_void_p(1)
    assert L.abx_query_spatial_1p(None, C.byref(pr), 4, None, 0, None, None, 0, info, None) == \
        abx.ERR_INVALID_ARG


def test_build_rejects_unknown_hierarchy():
    abx, L = _lib()
    tb, sb = C.c_size_t(), C.c_size_t()
    ok = abx.Primitives(abx.PRIM_POINTS, 1, 5)
    for h, want in ((0, abx.OK), (1, abx.OK), (2, abx.ERR_INVALID_ARG), (-1, abx.ERR_INVALID_ARG)):
        opt = abx.BuildOptions(abx.NODES_FP32, 21, h)
        assert L.abx_bvh_build_sizes(C.byref(ok), C.byref(opt), C.byref(tb), C.byref(sb)) == want


def test_build_node_order_option():
    abx, L = _lib()
    tb, sb = C.c_size_t(), C.c_size_t()
    ok = abx.Primitives(abx.PRIM_POINTS, 1, 5)
    cases = (
        (abx.NODES_Q16, 0, 0, abx.OK), (abx.NODES_Q16, 0, 1, abx.OK), (abx.NODES_Q16, 0, 2, abx.OK),
        (abx.NODES_FP32, 0, 2, abx.ERR_UNSUPPORTED),    # depth-first order needs Q16 nodes
        (abx.NODES_Q16, 1, 2, abx.ERR_UNSUPPORTED),     # and the Karras hierarchy
        (abx.NODES_Q16, 0, 3, abx.ERR_INVALID_ARG), (abx.NODES_Q16, 0, -1, abx.ERR_INVALID_ARG))
    for fmt, h, order, want in cases:
        opt = abx.BuildOptions(fmt, 21, h, order)
        assert L.abx_bvh_build_sizes(C.byref(ok), C.byref(opt), C.byref(tb), C.byref(sb)) == want, \
            (fmt, h, order)
    # the order's scratch is reserved only where it is used
    big = abx.Primitives(abx.PRIM_POINTS, 1, 1 << 20)
    sizes = []
    for order in (1, 2):
        opt = abx.BuildOptions(abx.NODES_Q16, 21, 0, order)
        assert L.abx_bvh_build_sizes(C.byref(big), C.byref(opt), C.byref(tb), C.byref(sb)) == abx.OK
        sizes.append(sb.value)
    assert sizes[1] - sizes[0] >= 16 * ((1 << 20) - 1)
