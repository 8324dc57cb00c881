"""Python binding of libabx (ctypes), argument marshalling only.

Every step of construction and search runs in the library's HIP kernels; this
module allocates device buffers with PyTorch (the library never allocates),
passes raw device pointers and the current HIP stream, and maps status codes
to exceptions.  If ``libabx.so`` is missing or cannot be loaded, every call
raises -- there is no fallback.

Entry points (same names as the C-ABI, ``abx_`` prefix dropped):

* ``bvh_build(prims, kind=None, node_format="fp32", morton_bits=21) -> BVH``
* ``query_spatial(bvh, data, radius=..., radii=None, predicate="within",
  sort_queries=True, capacity=None) -> (offsets, indices)``
* ``query_spatial_1p(bvh, data, buffer_size, ...) -> (offsets, indices, traversals)``
* ``query_nearest(bvh, points, k, sort_queries=True) -> (offsets, indices, distances)``
* ``query_spatial_stats`` / ``query_nearest_stats`` -> int32 [m, 2]
* ``morton_codes``, ``radix_sort_pairs`` (building blocks)
* ``timing_enable``, ``timing_reset``, ``timing_get``
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# ABX_LIBRARY: another build of the same library (the thread-sanitised
# build the tests make of the host code)
LIB_PATH = os.environ.get("ABX_LIBRARY") or os.path.join(_HERE, "libabx.so")

# status codes (include/abx.h)
(OK, ERR_INVALID_ARG, ERR_INVALID_INPUT, ERR_CAPACITY, ERR_OVERFLOW, ERR_HIP, ERR_UNSUPPORTED, PENDING,
 ERR_DEVICE) = range(9)
PRIM_POINTS, PRIM_BOXES = 0, 1
NODES_FP32, NODES_Q16, NODES_Q16W = 0, 1, 2
PRED_WITHIN, PRED_INTERSECTS_BOX = 0, 1

_FORMATS = {"fp32": NODES_FP32, "q16": NODES_Q16, "q16w": NODES_Q16W, NODES_FP32: NODES_FP32,
            NODES_Q16: NODES_Q16, NODES_Q16W: NODES_Q16W}
_HIERARCHIES = {"karras": 0, "agglomerative": 1}
_ORDERS = {"auto": 0, "build": 1, "depth_first": 2}
ORDER_BUILD, ORDER_DEPTH_FIRST = 1, 2
_PREDS = {"within": PRED_WITHIN, "intersects": PRED_INTERSECTS_BOX,
          PRED_WITHIN: PRED_WITHIN, PRED_INTERSECTS_BOX: PRED_INTERSECTS_BOX}


class AbxError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        msg = _lib().abx_status_string(status).decode() if _LIB is not None else str(status)
        extra = ""
        if status == ERR_HIP and _LIB is not None:
            extra = f" (hip error {_LIB.abx_last_hip_error()})"
        super().__init__(f"{where}: {msg}{extra}")


class Primitives(C.Structure):
    _fields_ = [("kind", C.c_int), ("data", C.c_void_p), ("n", C.c_int64)]


class BuildOptions(C.Structure):
    _fields_ = [("node_format", C.c_int), ("morton_bits", C.c_int32), ("hierarchy", C.c_int32),
                ("node_order", C.c_int32)]


class Predicates(C.Structure):
    _fields_ = [("kind", C.c_int), ("data", C.c_void_p), ("m", C.c_int64), ("radii", C.c_void_p),
                ("radius", C.c_float), ("sort_queries", C.c_int32)]


class ForestPrimitives(C.Structure):
    _fields_ = [("trees", C.c_int32), ("offsets_host", C.c_void_p), ("offsets_dev", C.c_void_p),
                ("data", C.c_void_p), ("node_format", C.c_int)]


class ForestQueries(C.Structure):
    _fields_ = [("offsets_host", C.c_void_p), ("offsets_dev", C.c_void_p), ("data", C.c_void_p)]


class ForestConfig(C.Structure):
    _fields_ = [("blocks_per_cu", C.c_int32), ("tiles_per_grab", C.c_int32), ("budget", C.c_int64)]


class ServerConfig(C.Structure):
    _fields_ = [("slots", C.c_int32), ("arena", C.c_void_p), ("arena_bytes", C.c_size_t),
                ("host_bytes", C.c_size_t), ("poll_us", C.c_int32), ("simulate", C.c_int32),
                ("sim_ns_per_query", C.c_double), ("merge_queries", C.c_int64),
                ("small_queries", C.c_int64), ("merge_large", C.c_int64)]


class Request(C.Structure):
    _fields_ = [("tree", C.c_int32), ("kind", C.c_int), ("queries", C.c_void_p), ("m", C.c_int64),
                ("radius", C.c_float), ("k", C.c_int32), ("t_arrival", C.c_double)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("m", C.c_int64), ("total", C.c_int64),
                ("offsets", C.c_void_p), ("indices", C.c_void_p), ("distances", C.c_void_p),
                ("t_arrival", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("t_device", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("queries", C.c_int64), ("max_in_flight", C.c_int64), ("in_flight", C.c_int64),
                ("queued", C.c_int64), ("device_high_water", C.c_size_t),
                ("host_high_water", C.c_size_t), ("requeued", C.c_int64), ("batches", C.c_int64)]


REQ_RADIUS, REQ_NEAREST = 0, 1


class Layout(C.Structure):
    _fields_ = [("n", C.c_int64), ("kind", C.c_int32), ("node_format", C.c_int32),
                ("morton_bits", C.c_int32), ("height", C.c_int32), ("hierarchy", C.c_int32),
                ("root", C.c_int32), ("node_order", C.c_int32), ("scene", C.c_float * 6),
                ("nodes_offset", C.c_size_t), ("node_bytes", C.c_size_t),
                ("leaves_offset", C.c_size_t), ("leaf_bytes", C.c_size_t),
                ("q16_origin", C.c_float * 3), ("q16_scale", C.c_float * 3),
                ("node_count", C.c_int64)]


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libabx.so not built ({LIB_PATH}); run "
                               "`python -m paper_1908_11807_amd.build` (needs ROCm hipcc)")
        L = C.CDLL(LIB_PATH)
        vp, sz, i64, i32 = C.c_void_p, C.c_size_t, C.c_int64, C.c_int32
        P = C.POINTER
        sig = {
            "abx_bvh_build_sizes": [P(Primitives), P(BuildOptions), P(sz), P(sz)],
            "abx_bvh_build": [P(Primitives), P(BuildOptions), vp, sz, vp, sz, vp, P(vp)],
            "abx_bvh_destroy": [vp],
            "abx_bvh_get_layout": [vp, P(Layout)],
            "abx_query_spatial_sizes": [vp, P(Predicates), P(sz)],
            "abx_query_spatial": [vp, P(Predicates), vp, sz, vp, vp, i64, P(i64), vp],
            "abx_query_spatial_fill": [vp, P(Predicates), vp, sz, vp, vp, i64, vp],
            "abx_query_spatial_1p_sizes": [vp, P(Predicates), i32, P(sz)],
            "abx_query_spatial_1p": [vp, P(Predicates), i32, vp, sz, vp, vp, i64, vp, vp],
            "abx_query_nearest_sizes": [vp, i64, i32, P(sz)],
            "abx_query_nearest": [vp, vp, i64, i32, i32, vp, sz, vp, vp, vp, vp],
            "abx_query_nearest_static": [vp, vp, i64, i32, i32, vp, vp, vp, vp],
            "abx_query_spatial_stats": [vp, P(Predicates), vp, sz, vp, vp],
            "abx_query_nearest_stats": [vp, vp, i64, i32, i32, vp, sz, vp, vp],
            "abx_morton_codes": [C.c_int, vp, i64, vp, i32, vp, vp],
            "abx_radix_sort_sizes": [i64, i32, P(sz)],
            "abx_radix_sort_pairs": [vp, vp, i64, i32, vp, vp, vp, sz, vp],
            "abx_radix_sort_check": [vp, i64, i32, vp],
            "abx_inject_fault": [i32, i64],
            "abx_timing_get": [C.c_char_p, P(C.c_double), P(i64)],
            "abx_forest_build_sizes": [P(ForestPrimitives), P(sz), P(sz)],
            "abx_forest_build": [P(ForestPrimitives), vp, sz, vp, sz, vp, P(vp)],
            "abx_forest_check": [vp, vp],
            "abx_forest_destroy": [vp],
            "abx_forest_query_nearest_sizes": [vp, P(ForestQueries), i32, P(sz), P(i64)],
            "abx_forest_query_nearest": [vp, P(ForestQueries), i32, P(ForestConfig), vp, sz, vp, vp,
                                         vp, vp],
            "abx_forest_autotune": [vp, P(ForestQueries), i32, vp, sz, vp, vp, vp, vp, C.c_char_p,
                                    P(ForestConfig)],
            "abx_forest_query_nearest_stats": [vp, P(ForestQueries), i32, vp, sz, vp, vp, vp],
            "abx_server_create": [P(ServerConfig), P(vp)],
            "abx_server_add_tree": [vp, vp, P(i32)],
            "abx_server_submit": [vp, P(Request), P(C.c_uint64)],
            "abx_server_poll": [vp, C.c_uint64, P(Result)],
            "abx_server_wait": [vp, C.c_uint64, P(Result)],
            "abx_server_release": [vp, C.c_uint64],
            "abx_server_drain": [vp],
            "abx_server_get_stats": [vp, P(ServerStats)],
            "abx_server_destroy": [vp],
            "abx_graph_begin": [vp],
            "abx_graph_end": [vp, P(vp)],
            "abx_graph_launch": [vp, vp],
            "abx_graph_destroy": [vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.abx_status_string.argtypes = [C.c_int]
        L.abx_status_string.restype = C.c_char_p
        L.abx_version.restype = C.c_char_p
        L.abx_last_hip_error.restype = C.c_int
        L.abx_server_now.restype = C.c_double
        L.abx_set_nearest_budget.argtypes = [C.c_int64]
        L.abx_set_nearest_budget.restype = C.c_int64
        L.abx_set_sort_spin_limit.argtypes = [C.c_int64]
        L.abx_set_sort_spin_limit.restype = C.c_int64
        L.abx_set_refit_table_probes.argtypes = [C.c_int64]
        L.abx_set_refit_table_probes.restype = C.c_int64
        L.abx_timing_enable.argtypes = [C.c_int]
        L.abx_timing_enable.restype = None
        L.abx_timing_reset.restype = None
        _LIB = L
    return _LIB


def library():
    """The loaded ctypes library (raises if it is not built)."""
    return _lib()


def _check(st, where):
    if st != OK:
        raise AbxError(st, where)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


def _dev_f32(x, width, what):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if x.dtype != torch.float32:
        raise TypeError(f"{what} must be float32")
    x = x.contiguous()
    if x.numel() % width:
        raise ValueError(f"{what} must have {width} columns")
    return x.view(-1, width)


def _bytes(n, device):
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


class BVH:
    """A built tree: the device tree buffer (torch) plus the library handle."""

    def __init__(self, handle, tree, prims, kind):
        self._h = handle
        self.tree = tree
        self.prims = prims      # keeps the primitives alive for the tree's lifetime
        self.kind = kind
        lay = Layout()
        _check(_lib().abx_bvh_get_layout(self._h, C.byref(lay)), "abx_bvh_get_layout")
        self.layout = lay

    @property
    def handle(self):
        return self._h

    @property
    def n(self):
        return int(self.layout.n)

    @property
    def height(self):
        return int(self.layout.height)

    @property
    def node_format(self):
        return int(self.layout.node_format)

    @property
    def scene(self):
        return list(self.layout.scene)

    def nodes_bytes(self):
        lay = self.layout
        return self.tree[lay.nodes_offset: lay.nodes_offset + int(lay.node_count) * lay.node_bytes]

    def leaves_bytes(self):
        lay = self.layout
        return self.tree[lay.leaves_offset: lay.leaves_offset + self.n * lay.leaf_bytes]

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _LIB is not None:
            _LIB.abx_bvh_destroy(h)


def bvh_build(prims, kind=None, node_format="fp32", morton_bits=21, hierarchy="karras",
              node_order="auto"):
    """Build the LBVH of ``prims`` (float32 CUDA tensor, [n,3] points or [n,6] boxes).

    ``hierarchy``: "karras" (per-node range search, then refit) or
    "agglomerative" (hierarchy and refit in one bottom-up pass).
    ``node_order``: "auto", "build" (the hierarchy's numbering) or
    "depth_first" (Q16 Karras trees)."""
    L = _lib()
    if kind is None:
        kind = PRIM_BOXES if (prims.dim() == 2 and prims.shape[-1] == 6) else PRIM_POINTS
    width = 3 if kind == PRIM_POINTS else 6
    p = _dev_f32(prims, width, "primitives")
    pr = Primitives(kind, p.data_ptr() if p.numel() else None, p.shape[0])
    opt = BuildOptions(_FORMATS[node_format], int(morton_bits), _HIERARCHIES[hierarchy],
                       _ORDERS[node_order])
    tb, sb = C.c_size_t(), C.c_size_t()
    _check(L.abx_bvh_build_sizes(C.byref(pr), C.byref(opt), C.byref(tb), C.byref(sb)),
           "abx_bvh_build_sizes")
    tree = _bytes(tb.value, p.device)
    scratch = _bytes(sb.value, p.device)
    h = C.c_void_p()
    _check(L.abx_bvh_build(C.byref(pr), C.byref(opt), _ptr(tree), tb.value, _ptr(scratch), sb.value,
                           _stream(), C.byref(h)), "abx_bvh_build")
    return BVH(h, tree, p, kind)


def _preds(data, predicate, radius, radii, sort_queries):
    kind = _PREDS[predicate]
    width = 3 if kind == PRED_WITHIN else 6
    d = _dev_f32(data, width, "query data")
    rr = None
    if radii is not None:
        rr = _dev_f32(radii, 1, "radii").view(-1)
        if rr.shape[0] != d.shape[0]:
            raise ValueError("radii must have one entry per query")
    pr = Predicates(kind, d.data_ptr() if d.numel() else None, d.shape[0],
                    rr.data_ptr() if rr is not None and rr.numel() else None,
                    float(radius if radius is not None else 0.0), 1 if sort_queries else 0)
    return pr, d, rr


def query_spatial(bvh, data, radius=None, radii=None, predicate="within", sort_queries=True,
                  capacity=None):
    """Spatial predicates -> CSR (offsets int32 [m+1], indices int32 [total]).

    Two-pass count-and-fill.  ``capacity`` is the caller's estimate of the
    total number of results (the paper's buffer_size); when it is missing or
    too small the exact total is allocated after the counting pass.
    """
    L = _lib()
    pr, d, rr = _preds(data, predicate, radius, radii, sort_queries)
    m = d.shape[0]
    sb = C.c_size_t()
    _check(L.abx_query_spatial_sizes(bvh.handle, C.byref(pr), C.byref(sb)), "abx_query_spatial_sizes")
    scratch = _bytes(sb.value, d.device)
    offsets = torch.empty(m + 1, dtype=torch.int32, device=d.device)
    cap = int(capacity or 0)
    indices = torch.empty(max(cap, 1), dtype=torch.int32, device=d.device)
    total = C.c_int64()
    st = L.abx_query_spatial(bvh.handle, C.byref(pr), _ptr(scratch), sb.value, _ptr(offsets),
                             _ptr(indices) if cap > 0 else C.c_void_p(0), cap, C.byref(total),
                             _stream())
    if st == ERR_CAPACITY:
        indices = torch.empty(max(total.value, 1), dtype=torch.int32, device=d.device)
        st = L.abx_query_spatial_fill(bvh.handle, C.byref(pr), _ptr(scratch), sb.value,
                                      _ptr(offsets), _ptr(indices), total.value, _stream())
    _check(st, "abx_query_spatial")
    return offsets, indices[: total.value]


def query_spatial_1p(bvh, data, buffer_size, radius=None, radii=None, predicate="within",
                     sort_queries=True, capacity=None):
    """One-pass spatial query -> (offsets, indices, traversals made).

    ``buffer_size`` is the per-query estimate of the hits (the paper's
    buffer_size): when no query exceeds it, one traversal answers the batch
    and the stored rows are compacted; otherwise the fill traversal of the
    two-pass scheme runs.  ``capacity`` (default m * buffer_size) sizes the
    index buffer; a larger total is allocated after reading it back.
    """
    L = _lib()
    pr, d, rr = _preds(data, predicate, radius, radii, sort_queries)
    m = d.shape[0]
    sb = C.c_size_t()
    _check(L.abx_query_spatial_1p_sizes(bvh.handle, C.byref(pr), int(buffer_size), C.byref(sb)),
           "abx_query_spatial_1p_sizes")
    scratch = _bytes(sb.value, d.device)
    offsets = torch.empty(m + 1, dtype=torch.int32, device=d.device)
    cap = int(capacity if capacity is not None else m * int(buffer_size))
    indices = torch.empty(max(cap, 1), dtype=torch.int32, device=d.device)
    info = torch.zeros(2, dtype=torch.int32, device=d.device)
    _check(L.abx_query_spatial_1p(bvh.handle, C.byref(pr), int(buffer_size), _ptr(scratch), sb.value,
                                  _ptr(offsets), _ptr(indices) if cap > 0 else C.c_void_p(0), cap,
                                  _ptr(info), _stream()), "abx_query_spatial_1p")
    st, passes = (int(v) for v in info.cpu().tolist())
    total = int(offsets[-1].item())
    if st == ERR_CAPACITY:
        indices = torch.empty(max(total, 1), dtype=torch.int32, device=d.device)
        _check(L.abx_query_spatial_fill(bvh.handle, C.byref(pr), _ptr(scratch), sb.value,
                                        _ptr(offsets), _ptr(indices), total, _stream()),
               "abx_query_spatial_fill")
        passes = 2
    else:
        _check(st, "abx_query_spatial_1p")
    return offsets, indices[:total], passes


def query_nearest(bvh, points, k, sort_queries=True):
    """k nearest primitives of each point -> (offsets, indices [m,k'], distances [m,k'])."""
    L = _lib()
    q = _dev_f32(points, 3, "query points")
    m = q.shape[0]
    kk = max(0, min(int(k), bvh.n))
    sb = C.c_size_t()
    _check(L.abx_query_nearest_sizes(bvh.handle, m, int(k), C.byref(sb)), "abx_query_nearest_sizes")
    scratch = _bytes(sb.value, q.device)
    offsets = torch.empty(m + 1, dtype=torch.int32, device=q.device)
    idx = torch.empty((m, kk), dtype=torch.int32, device=q.device)
    dist = torch.empty((m, kk), dtype=torch.float32, device=q.device)
    _check(L.abx_query_nearest(bvh.handle, _ptr(q), m, int(k), 1 if sort_queries else 0,
                               _ptr(scratch), sb.value, _ptr(offsets), _ptr(idx), _ptr(dist),
                               _stream()), "abx_query_nearest")
    return offsets, idx, dist


# scratch of abx_query_nearest_static, one library-owned array per GPU
STATIC_SCRATCH_BYTES = 64 << 20


def query_nearest_static(bvh, points, k, sort_queries=True, out=None):
    """The same query as ``query_nearest`` through the entry point that
    allocates nothing (its scratch is the library's per-GPU array).
    ``out`` = (offsets [m+1], indices [m,k'], distances [m,k']) to write
    into; otherwise they are allocated here, outside the library."""
    L = _lib()
    q = _dev_f32(points, 3, "query points")
    m = q.shape[0]
    kk = max(0, min(int(k), bvh.n))
    if out is None:
        out = (torch.empty(m + 1, dtype=torch.int32, device=q.device),
               torch.empty((m, kk), dtype=torch.int32, device=q.device),
               torch.empty((m, kk), dtype=torch.float32, device=q.device))
    offsets, idx, dist = out
    _check(L.abx_query_nearest_static(bvh.handle, _ptr(q), m, int(k), 1 if sort_queries else 0,
                                      _ptr(offsets), _ptr(idx), _ptr(dist), _stream()),
           "abx_query_nearest_static")
    return offsets, idx, dist


def query_spatial_stats(bvh, data, radius=None, radii=None, predicate="within", sort_queries=True):
    """Per query: (internal nodes visited, leaf records read), int32 [m, 2]."""
    L = _lib()
    pr, d, rr = _preds(data, predicate, radius, radii, sort_queries)
    sb = C.c_size_t()
    _check(L.abx_query_spatial_sizes(bvh.handle, C.byref(pr), C.byref(sb)), "abx_query_spatial_sizes")
    scratch = _bytes(sb.value, d.device)
    stats = torch.empty((d.shape[0], 2), dtype=torch.int32, device=d.device)
    _check(L.abx_query_spatial_stats(bvh.handle, C.byref(pr), _ptr(scratch), sb.value, _ptr(stats),
                                     _stream()), "abx_query_spatial_stats")
    return stats


def query_nearest_stats(bvh, points, k, sort_queries=True):
    L = _lib()
    q = _dev_f32(points, 3, "query points")
    sb = C.c_size_t()
    _check(L.abx_query_nearest_sizes(bvh.handle, q.shape[0], int(k), C.byref(sb)),
           "abx_query_nearest_sizes")
    scratch = _bytes(sb.value, q.device)
    stats = torch.empty((q.shape[0], 2), dtype=torch.int32, device=q.device)
    _check(L.abx_query_nearest_stats(bvh.handle, _ptr(q), q.shape[0], int(k),
                                     1 if sort_queries else 0, _ptr(scratch), sb.value,
                                     _ptr(stats), _stream()), "abx_query_nearest_stats")
    return stats


def morton_codes(prims, scene, bits, kind=None):
    """Morton codes (int64 tensor holding the uint64 codes) against a scene box."""
    L = _lib()
    if kind is None:
        kind = PRIM_BOXES if prims.shape[-1] == 6 else PRIM_POINTS
    p = _dev_f32(prims, 3 if kind == PRIM_POINTS else 6, "primitives")
    sc = _dev_f32(scene, 6, "scene").view(-1)
    codes = torch.empty(p.shape[0], dtype=torch.int64, device=p.device)
    _check(L.abx_morton_codes(kind, _ptr(p), p.shape[0], _ptr(sc), int(bits), _ptr(codes), _stream()),
           "abx_morton_codes")
    return codes


def radix_sort_pairs(keys, key_bits, vals=None, check=True):
    """Stable radix sort of (key, value) pairs; keys int32 (<=32 bits) or int64.
    With ``check`` the host waits for the sort and raises AbxError
    (ERR_DEVICE) if a tile gave up waiting for its predecessors."""
    L = _lib()
    n = keys.numel()
    keys = keys.contiguous()
    sb = C.c_size_t()
    _check(L.abx_radix_sort_sizes(n, int(key_bits), C.byref(sb)), "abx_radix_sort_sizes")
    scratch = _bytes(sb.value, keys.device)
    kout = torch.empty_like(keys)
    vout = torch.empty(n, dtype=torch.int32, device=keys.device)
    vin = None if vals is None else vals.contiguous()
    _check(L.abx_radix_sort_pairs(_ptr(keys), _ptr(vin), n, int(key_bits), _ptr(kout), _ptr(vout),
                                  _ptr(scratch), sb.value, _stream()), "abx_radix_sort_pairs")
    if check:
        _check(L.abx_radix_sort_check(_ptr(scratch), n, int(key_bits), _stream()),
               "abx_radix_sort_check")
    return kout, vout


FAULT_LAUNCH, FAULT_HOST_ALLOC = 0, 1


def inject_fault(kind, skip=0):
    """Test hook: the (skip + 1)-th next event of ``kind`` fails once as a HIP
    failure would (FAULT_LAUNCH: a kernel launch or a simulated server
    phase; FAULT_HOST_ALLOC: a server's pinned host arena); skip < 0
    disarms."""
    _check(_lib().abx_inject_fault(int(kind), int(skip)), "abx_inject_fault")


def set_sort_spin_limit(polls):
    """Polls of an unpublished predecessor before a sort tile gives up
    (< 0 restores the default; 0 forces the give-up, for tests).  Returns the
    previous value."""
    return int(_lib().abx_set_sort_spin_limit(int(polls)))


def set_refit_table_probes(probes):
    """Probes of the refit's LDS table per node before a pass climbs through
    global memory instead (< 0 restores the default, 0 always uses global
    memory; the tree is the same).  Returns the previous value."""
    return int(_lib().abx_set_refit_table_probes(int(probes)))


class ForestPlan:
    """A batched forest (section 2.2 batched mode across trees) with every
    device buffer allocated up front, so that the build and the query can be
    replayed eagerly or captured once in a HIP graph and replayed.

    points: float32 CUDA [N, 3]; offsets: int sequence [T+1] (tree t owns
    rows offsets[t]..offsets[t+1]); queries/query_offsets likewise; k <= 32.
    Results (after run() or a replay): self.offsets int32 [M+1],
    self.indices int32 [total] (tree-local), self.distances float32 [total].
    """

    def __init__(self, points, offsets, queries, query_offsets, k, node_format="q16"):
        import numpy as np
        L = _lib()
        self.k = int(k)
        self.points = _dev_f32(points, 3, "points")
        self.queries = _dev_f32(queries, 3, "queries")
        dev = self.points.device
        self._off_h = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        self._qoff_h = np.ascontiguousarray(np.asarray(query_offsets, dtype=np.int64))
        self.trees = self._off_h.shape[0] - 1
        if self._qoff_h.shape[0] != self.trees + 1:
            raise ValueError("query_offsets must have one entry per tree plus one")
        self._off_d = torch.from_numpy(self._off_h).to(dev)
        self._qoff_d = torch.from_numpy(self._qoff_h).to(dev)
        self._prims = ForestPrimitives(self.trees, self._off_h.ctypes.data, self._off_d.data_ptr(),
                                       self.points.data_ptr() if self.points.numel() else None,
                                       _FORMATS[node_format])
        self._q = ForestQueries(self._qoff_h.ctypes.data, self._qoff_d.data_ptr(),
                                self.queries.data_ptr() if self.queries.numel() else None)
        tb, sb = C.c_size_t(), C.c_size_t()
        _check(L.abx_forest_build_sizes(C.byref(self._prims), C.byref(tb), C.byref(sb)),
               "abx_forest_build_sizes")
        self.tree = _bytes(tb.value, dev)
        self._bscratch = _bytes(sb.value, dev)
        self._tb, self._sb = tb.value, sb.value
        self._h = None
        self.build()                      # the handle (host metadata) exists from here on
        qs, tot = C.c_size_t(), C.c_int64()
        _check(L.abx_forest_query_nearest_sizes(self._h, C.byref(self._q), self.k, C.byref(qs),
                                                C.byref(tot)), "abx_forest_query_nearest_sizes")
        self._qscratch = _bytes(qs.value, dev)
        self._qs = qs.value
        self.total = tot.value
        M = int(self._qoff_h[-1])
        self.offsets = torch.empty(M + 1, dtype=torch.int32, device=dev)
        self.indices = torch.empty(max(self.total, 1), dtype=torch.int32, device=dev)
        self.distances = torch.empty(max(self.total, 1), dtype=torch.float32, device=dev)
        self.config = None
        self._graph = None

    def build(self):
        L = _lib()
        h = C.c_void_p()
        _check(L.abx_forest_build(C.byref(self._prims), _ptr(self.tree), self._tb, _ptr(self._bscratch),
                                  self._sb, _stream(), C.byref(h)), "abx_forest_build")
        if self._h:
            cfg = getattr(self, "config", None)
            L.abx_forest_destroy(self._h)
            self._h = h
            if cfg is not None:
                self.config = cfg
        else:
            self._h = h

    def check(self):
        _check(_lib().abx_forest_check(self._h, _stream()), "abx_forest_check")

    def query(self, config=None):
        cfg = None
        if config is not None:
            cfg = ForestConfig(int(config["blocks_per_cu"]), int(config["tiles_per_grab"]),
                               int(config["budget"]))
        elif self.config is not None:
            c = self.config
            cfg = ForestConfig(c["blocks_per_cu"], c["tiles_per_grab"], c["budget"])
        _check(_lib().abx_forest_query_nearest(self._h, C.byref(self._q), self.k,
                                               C.byref(cfg) if cfg is not None else None,
                                               _ptr(self._qscratch), self._qs, _ptr(self.offsets),
                                               _ptr(self.indices), _ptr(self.distances), _stream()),
               "abx_forest_query_nearest")

    def run(self):
        self.build()
        self.query()
        return self.results()

    def results(self):
        t = self.total
        return self.offsets, self.indices[:t], self.distances[:t]

    def stats(self):
        """Per query (node visits, leaf records read), int32 [M, 2], caller's
        order: the same walks counted, one lane per query."""
        M = int(self._qoff_h[-1])
        st = torch.empty((M, 2), dtype=torch.int32, device=self.offsets.device)
        off = torch.empty(M + 1, dtype=torch.int32, device=self.offsets.device)
        _check(_lib().abx_forest_query_nearest_stats(self._h, C.byref(self._q), self.k, _ptr(self._qscratch),
                                                     self._qs, _ptr(off), _ptr(st), _stream()),
               "abx_forest_query_nearest_stats")
        return st

    def autotune(self, json_path=None):
        best = ForestConfig()
        _check(_lib().abx_forest_autotune(self._h, C.byref(self._q), self.k, _ptr(self._qscratch),
                                          self._qs, _ptr(self.offsets), _ptr(self.indices),
                                          _ptr(self.distances), _stream(),
                                          json_path.encode() if json_path else None, C.byref(best)),
               "abx_forest_autotune")
        self.config = dict(blocks_per_cu=best.blocks_per_cu, tiles_per_grab=best.tiles_per_grab,
                           budget=best.budget)
        return self.config

    def capture(self, build=True):
        """Capture (build +) query on the current stream (must not be the
        null stream) into a HIP graph; replay with replay()."""
        L = _lib()
        _check(L.abx_graph_begin(_stream()), "abx_graph_begin")
        try:
            if build:
                h2 = C.c_void_p()
                st = L.abx_forest_build(C.byref(self._prims), _ptr(self.tree), self._tb,
                                        _ptr(self._bscratch), self._sb, _stream(), C.byref(h2))
                if h2:
                    L.abx_forest_destroy(h2)   # host metadata only; self._h describes the same tree
                _check(st, "abx_forest_build")
            self.query()
        finally:
            g = C.c_void_p()
            st = L.abx_graph_end(_stream(), C.byref(g))
        _check(st, "abx_graph_end")
        if self._graph:
            L.abx_graph_destroy(self._graph)
        self._graph = g

    def replay(self):
        _check(_lib().abx_graph_launch(self._graph, _stream()), "abx_graph_launch")

    def __del__(self):
        if _LIB is None:
            return
        if getattr(self, "_graph", None):
            _LIB.abx_graph_destroy(self._graph)
        if getattr(self, "_h", None):
            _LIB.abx_forest_destroy(self._h)


def server_now():
    """Seconds on the server's steady clock (request arrival timestamps)."""
    return float(_lib().abx_server_now())


class Server:
    """Continuous-batching request server over device-resident trees.

    slots: concurrent batches (one HIP stream each); budget_bytes: the HBM
    arena for in-flight request data (allocated here with PyTorch and handed
    to the library); host_bytes: pinned host result arena (allocated by the
    library); merge_queries / small_queries / merge_large: merge limits and
    size classes (0: the library's defaults; a negative merge limit turns
    that merging off).  simulate=True runs the scheduler without the GPU.
    """

    def __init__(self, slots=4, budget_bytes=1 << 30, host_bytes=1 << 30, simulate=False,
                 sim_ns_per_query=0.0, poll_us=0, device="cuda", merge_queries=0, small_queries=0,
                 merge_large=0):
        L = _lib()
        self.arena = None if simulate else torch.empty(int(budget_bytes), dtype=torch.uint8, device=device)
        cfg = ServerConfig(int(slots), self.arena.data_ptr() if self.arena is not None else None,
                           int(budget_bytes), int(host_bytes), int(poll_us), 1 if simulate else 0,
                           float(sim_ns_per_query), int(merge_queries), int(small_queries),
                           int(merge_large))
        h = C.c_void_p()
        _check(L.abx_server_create(C.byref(cfg), C.byref(h)), "abx_server_create")
        self._h = h
        self._trees = []
        self._inputs = {}

    def add_tree(self, bvh):
        tid = C.c_int32()
        _check(_lib().abx_server_add_tree(self._h, bvh.handle if bvh is not None else None,
                                          C.byref(tid)), "abx_server_add_tree")
        self._trees.append(bvh)
        return tid.value

    def submit(self, tree, kind, queries, radius=0.0, k=0, t_arrival=None):
        """queries: host float32 [m, 3] (numpy or CPU tensor; pinned is fastest).
        Returns a ticket."""
        if isinstance(queries, torch.Tensor):
            if queries.is_cuda:
                raise TypeError("server queries are host memory")
            q = queries.contiguous()
            ptr, m = (q.data_ptr() if q.numel() else None), q.numel() // 3
        else:
            import numpy as np
            q = np.ascontiguousarray(queries, dtype=np.float32)
            ptr, m = (q.ctypes.data if q.size else None), q.size // 3
        req = Request(int(tree), int(kind), ptr, int(m), float(radius), int(k),
                      float(server_now() if t_arrival is None else t_arrival))
        t = C.c_uint64()
        _check(_lib().abx_server_submit(self._h, C.byref(req), C.byref(t)), "abx_server_submit")
        self._inputs[t.value] = q
        return t.value

    def _result(self, r, copy):
        import numpy as np
        out = dict(status=r.status, m=r.m, total=r.total, t_arrival=r.t_arrival,
                   t_admit=r.t_admit, t_done=r.t_done, t_device=r.t_device)
        if r.status == OK and copy:
            def arr(ptr, n, ct, dt):
                if not ptr or n == 0:
                    return np.zeros(0, dt)
                return np.ctypeslib.as_array(C.cast(ptr, C.POINTER(ct)), shape=(n,)).copy()
            out["offsets"] = arr(r.offsets, r.m + 1, C.c_int32, np.int32)
            out["indices"] = arr(r.indices, r.total, C.c_int32, np.int32)
            out["distances"] = arr(r.distances, r.total, C.c_float, np.float32) if r.distances else None
        return out

    def poll(self, ticket, copy=True):
        r = Result()
        st = _lib().abx_server_poll(self._h, ticket, C.byref(r))
        if st == PENDING:
            return None
        _check(st, "abx_server_poll")
        return self._result(r, copy)

    def wait(self, ticket, copy=True):
        r = Result()
        _check(_lib().abx_server_wait(self._h, ticket, C.byref(r)), "abx_server_wait")
        return self._result(r, copy)

    def release(self, ticket):
        _check(_lib().abx_server_release(self._h, ticket), "abx_server_release")
        self._inputs.pop(ticket, None)

    def drain(self):
        _check(_lib().abx_server_drain(self._h), "abx_server_drain")

    def stats(self):
        st = ServerStats()
        _check(_lib().abx_server_get_stats(self._h, C.byref(st)), "abx_server_get_stats")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            _lib().abx_server_destroy(self._h)
            self._h = None

    def __del__(self):
        if _LIB is not None:
            self.close()


def set_nearest_budget(visits):
    """Node visits before a nearest query moves to the cooperative (one
    workgroup per query) pass; <= 0 keeps every query on one lane.  Returns
    the previous value."""
    return int(_lib().abx_set_nearest_budget(int(visits)))


def timing_enable(on=True):
    _lib().abx_timing_enable(1 if on else 0)


def timing_reset():
    _lib().abx_timing_reset()


def timing_get(name):
    """(milliseconds summed, launches) of kernels called ``name`` since the last reset."""
    ms, cnt = C.c_double(), C.c_int64()
    _check(_lib().abx_timing_get(name.encode(), C.byref(ms), C.byref(cnt)), "abx_timing_get")
    return ms.value, cnt.value


def version():
    return _lib().abx_version().decode()
