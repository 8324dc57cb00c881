"""CPU oracle for the LBVH search path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The product library never calls it
and shares no code with it: the arithmetic lives in ``oracle.c`` (plain C,
double precision distances, brute force), wrapped here with ctypes and
numpy.  See the header of ``oracle.c`` for the paper passages each function
follows.

Exported (numpy in, numpy out):

* ``scene_box(prims, kind)``                  -> (box[6] float32, bad: bool)
* ``morton(prims, kind, scene, bits)``        -> uint64 codes
* ``sort_codes(codes)``                       -> (sorted codes, perm)   stable
* ``hierarchy(sorted_codes, keybits)``        -> (child_kind, child_index, range)
* ``refit(prims, kind, perm, child_kind, child_index)`` -> boxes [n-1, 6]
* ``build(prims, kind, bits)``                -> dict with all of the above
* ``spatial(prims, kind, queries, pred, radius | radii)`` -> (offsets, indices)
* ``nearest(prims, kind, queries, k)``        -> (indices [m, k'], dist [m, k'])
* ``distances(prims, kind, q, sel)``          -> float64 distances
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

POINTS, BOXES = 0, 1
WITHIN, INTERSECTS = 0, 1

_lib = None


def build_library(force: bool = False) -> str:
    """Compile ``oracle.c`` with gcc into ``liboracle.so`` (no fused multiply-add)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _L():
    global _lib
    if _lib is None:
        build_library()
        lib = C.CDLL(_LIB_PATH)
        p = C.c_void_p
        i64 = C.c_int64
        ci = C.c_int
        lib.oracle_scene_box.argtypes = [p, i64, ci, p]
        lib.oracle_scene_box.restype = ci
        lib.oracle_morton.argtypes = [p, i64, ci, p, ci, p]
        lib.oracle_hierarchy.argtypes = [p, i64, ci, p, p, p]
        lib.oracle_refit.argtypes = [p, ci, p, i64, p, p, p]
        lib.oracle_spatial_count.argtypes = [p, i64, ci, ci, p, i64, p, C.c_float, p]
        lib.oracle_spatial_fill.argtypes = [p, i64, ci, ci, p, i64, p, C.c_float, p, p]
        lib.oracle_nearest.argtypes = [p, i64, ci, p, i64, i64, p, p]
        lib.oracle_distances.argtypes = [p, ci, p, p, i64, p]
        lib.oracle_num_threads.restype = ci
        lib.oracle_set_num_threads.argtypes = [ci]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _prims(prims, kind):
    a = np.ascontiguousarray(prims, dtype=np.float32)
    w = 3 if kind == POINTS else 6
    if a.ndim != 2 or a.shape[1] != w:
        a = a.reshape(-1, w)
    return a


def num_threads() -> int:
    return _L().oracle_num_threads()


def set_num_threads(t: int) -> None:
    _L().oracle_set_num_threads(int(t))


def scene_box(prims, kind=POINTS):
    p = _prims(prims, kind)
    out = np.zeros(6, np.float32)
    bad = _L().oracle_scene_box(_ptr(p), p.shape[0], kind, _ptr(out))
    return out, bool(bad)


def morton(prims, kind, scene, bits):
    p = _prims(prims, kind)
    s = np.ascontiguousarray(scene, dtype=np.float32)
    out = np.zeros(p.shape[0], np.uint64)
    _L().oracle_morton(_ptr(p), p.shape[0], kind, _ptr(s), int(bits), _ptr(out))
    return out


def sort_codes(codes):
    """Stable sort of the codes (ties keep input order); returns (sorted, perm)."""
    perm = np.argsort(codes, kind="stable").astype(np.int64)
    return codes[perm], perm


def hierarchy(sorted_codes, keybits):
    c = np.ascontiguousarray(sorted_codes, dtype=np.uint64)
    n = c.shape[0]
    ni = max(n - 1, 0)
    kind = np.zeros(2 * ni, np.int8)
    idx = np.zeros(2 * ni, np.int64)
    rng = np.zeros(2 * ni, np.int64)
    _L().oracle_hierarchy(_ptr(c), n, int(keybits), _ptr(kind), _ptr(idx), _ptr(rng))
    return kind.reshape(ni, 2), idx.reshape(ni, 2), rng.reshape(ni, 2)


def refit(prims, kind, perm, child_kind, child_index):
    p = _prims(prims, kind)
    n = p.shape[0]
    ni = max(n - 1, 0)
    boxes = np.zeros((ni, 6), np.float32)
    perm = np.ascontiguousarray(perm, dtype=np.int64)
    ck = np.ascontiguousarray(child_kind, dtype=np.int8)
    ci = np.ascontiguousarray(child_index, dtype=np.int64)
    _L().oracle_refit(_ptr(p), kind, _ptr(perm), n, _ptr(ck), _ptr(ci), _ptr(boxes))
    return boxes


def build(prims, kind=POINTS, bits=21):
    """The whole construction of section 2.1, step by step."""
    scene, bad = scene_box(prims, kind)
    codes = morton(prims, kind, scene, bits)
    sc, perm = sort_codes(codes)
    ck, ci, rg = hierarchy(sc, 3 * bits)
    boxes = refit(prims, kind, perm, ck, ci)
    return dict(scene=scene, bad=bad, codes=codes, sorted_codes=sc, perm=perm,
                child_kind=ck, child_index=ci, range=rg, boxes=boxes)


def spatial(prims, kind, queries, pred=WITHIN, radius=0.0, radii=None):
    """CSR (offsets int64 [m+1], indices int64) of a batch of spatial predicates."""
    p = _prims(prims, kind)
    qw = 3 if pred == WITHIN else 6
    q = np.ascontiguousarray(queries, dtype=np.float32).reshape(-1, qw)
    m = q.shape[0]
    rr = None if radii is None else np.ascontiguousarray(radii, dtype=np.float32)
    counts = np.zeros(m, np.int64)
    L = _L()
    L.oracle_spatial_count(_ptr(p), p.shape[0], kind, pred, _ptr(q), m, _ptr(rr),
                           float(np.float32(radius)), _ptr(counts))
    offsets = np.zeros(m + 1, np.int64)
    np.cumsum(counts, out=offsets[1:])
    indices = np.zeros(int(offsets[-1]), np.int64)
    L.oracle_spatial_fill(_ptr(p), p.shape[0], kind, pred, _ptr(q), m, _ptr(rr),
                          float(np.float32(radius)), _ptr(offsets), _ptr(indices))
    return offsets, indices


def nearest(prims, kind, queries, k):
    """Rows of the min(k, n) nearest primitives, by (distance, index)."""
    p = _prims(prims, kind)
    q = np.ascontiguousarray(queries, dtype=np.float32).reshape(-1, 3)
    n, m = p.shape[0], q.shape[0]
    kk = max(0, min(int(k), n))
    idx = np.zeros((m, kk), np.int64)
    dist = np.zeros((m, kk), np.float64)
    if kk > 0 and m > 0:
        _L().oracle_nearest(_ptr(p), n, kind, _ptr(q), m, int(k), _ptr(idx), _ptr(dist))
    return idx, dist


def distances(prims, kind, q, sel=None):
    p = _prims(prims, kind)
    qq = np.ascontiguousarray(q, dtype=np.float32).reshape(3)
    s = None if sel is None else np.ascontiguousarray(sel, dtype=np.int64)
    cnt = p.shape[0] if s is None else s.shape[0]
    out = np.zeros(cnt, np.float64)
    _L().oracle_distances(_ptr(p), kind, _ptr(qq), _ptr(s), cnt, _ptr(out))
    return out
