"""GPU parity: every kernel and every entry point of libabx against the CPU
oracle, on seeded inputs that span several tiles and a ragged tail, plus the
edge cases of the method.  Runs only on an MI355X (marker `gpu`)."""
import numpy as np
import pytest
import torch

from paper_1908_11807_amd import abx, datagen
from parity import check_nearest, check_spatial, decode_tree, dequantise

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# ----------------------------------------------------------- building blocks

@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("bits", [10, 21])
def test_morton_codes_bit_exact(orc, kind, bits):
    pts = datagen.clusters(20_011, 3)
    prims = pts if kind == 0 else datagen.boxes_around(pts, 4, 0.01)
    scene, _ = orc.scene_box(prims, kind)
    want = orc.morton(prims, kind, scene, bits)
    got = host(abx.morton_codes(dev(prims), dev(scene), bits, kind=kind)).view(np.uint64)
    assert np.array_equal(got, want)


# tiles of 5120 32-bit and 5376 64-bit keys: one tile exactly, a key either
# side, two tiles and a ragged third
@pytest.mark.parametrize("n", [1, 2, 4095, 4096, 5119, 5120, 5121, 5375, 5376, 5377, 10_753,
                               15_361, 100_003])
@pytest.mark.parametrize("key_bits", [30, 63])
def test_radix_sort_stable(n, key_bits):
    rng = np.random.default_rng(n + key_bits)
    # few distinct keys so that stability is exercised
    keys = rng.integers(0, 2 ** 12, size=n).astype(np.uint64) << np.uint64(key_bits - 12)
    keys |= rng.integers(0, 3, size=n).astype(np.uint64)
    if key_bits <= 32:
        k = dev(keys.astype(np.uint32).view(np.int32))
    else:
        k = dev(keys.view(np.int64))
    ko, vo = abx.radix_sort_pairs(k, key_bits)
    perm = np.argsort(keys, kind="stable")
    assert np.array_equal(host(vo), perm)
    got_keys = host(ko).view(np.uint32 if key_bits <= 32 else np.uint64).astype(np.uint64)
    assert np.array_equal(got_keys, keys[perm])


def test_radix_sort_with_values():
    rng = np.random.default_rng(5)
    n = 50_000
    keys = rng.integers(0, 2 ** 30, size=n).astype(np.uint32)
    vals = rng.integers(-1000, 1000, size=n).astype(np.int32)
    ko, vo = abx.radix_sort_pairs(dev(keys.view(np.int32)), 30, vals=dev(vals))
    perm = np.argsort(keys, kind="stable")
    assert np.array_equal(host(vo), vals[perm])


# ---------------------------------------------------------------- construction

def _check_tree_vs_oracle(orc, prims, kind, bits, fmt, node_order="auto"):
    t = abx.bvh_build(dev(prims), kind=kind, node_format=fmt, morton_bits=bits, node_order=node_order)
    if node_order == "depth_first":
        assert t.layout.node_order == abx.ORDER_DEPTH_FIRST
    ref = orc.build(prims, kind, bits)
    n = prims.shape[0]
    got = decode_tree(t)
    assert np.array_equal(got["perm"], ref["perm"])
    np.testing.assert_array_equal(np.array(t.scene, np.float32), ref["scene"])
    if n >= 2:
        assert np.array_equal(got["child_kind"], ref["child_kind"])
        assert np.array_equal(got["child_index"], ref["child_index"])
    # node boxes: exact unions (FP32) / outward containment (Q16)
    ni = max(n - 1, 0)
    if ni:
        child_box = np.empty((ni, 2, 6), np.float32)
        ck, ci = ref["child_kind"], ref["child_index"]
        sp = np.asarray(prims, np.float32).reshape(n, -1)[ref["perm"]]
        leafbox = np.concatenate([sp[:, :3], sp[:, :3]], axis=1) if kind == 0 else sp
        for s in range(2):
            child_box[:, s] = np.where((ck[:, s] == 0)[:, None], leafbox[np.where(ck[:, s] == 0, ci[:, s], 0)],
                                       ref["boxes"][np.where(ck[:, s] == 1, ci[:, s], 0)])
        if fmt == "fp32":
            np.testing.assert_array_equal(got["boxes_l"], child_box[:, 0])
            np.testing.assert_array_equal(got["boxes_r"], child_box[:, 1])
        else:
            lay = t.layout
            for s, key in ((0, "q_l"), (1, "q_r")):
                d = dequantise(got[key], list(lay.q16_origin), list(lay.q16_scale))
                q = ck[:, s] == 1 if kind == 0 else np.ones(ni, bool)   # quantised slots
                assert np.all(d[q, :3] <= child_box[q, s, :3]), "q16 lower corner not outward"
                assert np.all(d[q, 3:] >= child_box[q, s, 3:]), "q16 upper corner not outward"
                # and the tightest such codes: one step inward leaves the box
                code = got[key].astype(np.int64)
                up = dequantise(np.minimum(code + 1, 65535), list(lay.q16_origin), list(lay.q16_scale))
                down = dequantise(np.maximum(code - 1, 0), list(lay.q16_origin), list(lay.q16_scale))
                flat = np.asarray(list(lay.q16_scale), np.float32) == 0   # one code per axis
                lo_ok = flat | (code[:, :3] == 65535) | (up[:, :3] > child_box[:, s, :3])
                hi_ok = flat | (code[:, 3:] == 0) | (down[:, 3:] < child_box[:, s, 3:])
                assert np.all(lo_ok[q]), "q16 lower corner not the tightest code"
                assert np.all(hi_ok[q]), "q16 upper corner not the tightest code"
    if fmt == "q16":
        sp = np.asarray(prims, np.float32).reshape(n, -1)[ref["perm"]]
        leafbox = np.concatenate([sp[:, :3], sp[:, :3]], axis=1) if kind == 0 else sp
        np.testing.assert_array_equal(got["leaf_boxes"], leafbox)
    return t


@pytest.mark.parametrize("n", [1, 2, 3, 17, 1000, 4097, 10_000])
@pytest.mark.parametrize("bits", [10, 21])
def test_build_points_matches_oracle(orc, n, bits):
    _check_tree_vs_oracle(orc, datagen.uniform_cube(n, 100 + n), 0, bits, "fp32")


@pytest.mark.parametrize("fmt,order", [("fp32", "auto"), ("q16", "build"), ("q16", "depth_first")])
@pytest.mark.parametrize("kind", [0, 1])
def test_build_formats_and_kinds(orc, fmt, order, kind):
    pts = datagen.clusters(12_345, 9)
    prims = pts if kind == 0 else datagen.boxes_around(pts, 10, 0.003)
    _check_tree_vs_oracle(orc, prims, kind, 21, fmt, order)


@pytest.mark.parametrize("n", [2, 3, 4, 1000, 8193])
def test_build_depth_first_small(orc, n):
    # depth-first node order down to the smallest trees (root 0, one node)
    _check_tree_vs_oracle(orc, datagen.uniform_cube(n, 300 + n), 0, 21, "q16", "depth_first")


@pytest.mark.parametrize("kind,fmt,order", [(0, "fp32", "auto"), (1, "q16", "auto"), (0, "q16", "depth_first")])
def test_build_all_refit_phases(orc, kind, fmt, order):
    # 1.3e6 leaves: 635 chunks of 2048 in 10 groups of 64 (the last one
    # ragged), so the in-chunk, in-group and cross-group refit phases all run
    pts = datagen.shell(1_300_000, 77, 0.99, 1.01)
    prims = pts if kind == 0 else datagen.boxes_around(pts, 78, 0.001)
    t = _check_tree_vs_oracle(orc, prims, kind, 21, fmt, order)
    assert t.height >= 2


@pytest.mark.parametrize("n", [2047, 2048, 2049, 4097, 131_071, 131_072, 131_073, 133_121, 262_145])
@pytest.mark.parametrize("fmt,order", [("fp32", "auto"), ("q16", "depth_first")])
def test_build_group_edges(orc, n, fmt, order):
    # chunks of 2048 leaves in groups of 64: one chunk or group exactly, one
    # leaf either side, one leaf past the first chunk of the second group, and
    # one past two groups; the in-group pass runs past 2048 leaves and the
    # top pass past 131 072
    _check_tree_vs_oracle(orc, datagen.clusters(n, 90), 0, 21, fmt, order)


@pytest.mark.parametrize("n", [2049, 131_073, 300_001, 1_000_000])
def test_refit_table_and_global_climbs_agree(n):
    # Above the 2048-leaf chunks the refit climbs in an LDS table; with no
    # probes every pass climbs through global memory, with one probe some
    # passes give up on the table midway.  The trees must not differ.
    pts = datagen.shell(n, 93)
    got = {}
    for probes in (-1, 0, 1):
        prev = abx.set_refit_table_probes(probes)
        try:
            for fmt in ("fp32", "q16"):
                t = abx.bvh_build(dev(pts), node_format=fmt)
                torch.cuda.synchronize()
                got[probes, fmt] = (t.height, t.nodes_bytes().cpu(), t.leaves_bytes().cpu())
                del t
        finally:
            abx.set_refit_table_probes(prev)
    for fmt in ("fp32", "q16"):
        h, nb, lb = got[-1, fmt]
        for probes in (0, 1):
            h2, nb2, lb2 = got[probes, fmt]
            assert h2 == h and torch.equal(nb2, nb) and torch.equal(lb2, lb), (fmt, probes)


def test_build_duplicates_and_degenerate_axis(orc):
    rng = np.random.default_rng(1)
    pts = rng.integers(0, 4, size=(3000, 3)).astype(np.float32)   # heavy duplicates
    pts[:, 2] = 0.5                                                # zero-extent axis
    for bits in (10, 21):
        for fmt in ("fp32", "q16"):
            _check_tree_vs_oracle(orc, pts, 0, bits, fmt)


def test_build_fig1(orc):
    leaves = np.array([[0.9, 0.25, 0, 1.04, 0.43, 0], [0.16, 0.2, 0, 0.30, 0.38, 0],
                       [0.6, 0.9, 0, 0.74, 1.08, 0], [0.2, 0.7, 0, 0.34, 0.88, 0],
                       [0.7, 0.2, 0, 0.84, 0.38, 0], [0, 0.1, 0, 0.14, 0.28, 0],
                       [0.5, 0.4, 0, 0.64, 0.58, 0], [0.8, 0.7, 0, 0.94, 0.88, 0]], np.float32)
    for bits in (10, 21):
        _check_tree_vs_oracle(orc, leaves, 1, bits, "fp32")


def test_build_rejects_nan_and_inverted(orc):
    p = datagen.uniform_cube(100, 1)
    p[50, 1] = np.nan
    with pytest.raises(abx.AbxError) as e:
        abx.bvh_build(dev(p))
    assert e.value.status == abx.ERR_INVALID_INPUT
    b = datagen.boxes_around(datagen.uniform_cube(100, 2), 3, 0.1)
    b[7, 0], b[7, 3] = b[7, 3], b[7, 0] - 1
    with pytest.raises(abx.AbxError) as e:
        abx.bvh_build(dev(b), kind=1)
    assert e.value.status == abx.ERR_INVALID_INPUT


def test_build_height_bound(orc):
    t = abx.bvh_build(dev(datagen.uniform_cube(10_000, 3)))
    ref = orc.build(datagen.uniform_cube(10_000, 3), 0, 21)
    # height = longest root-to-leaf path of the oracle's tree
    ck, ci = ref["child_kind"], ref["child_index"]
    depth = {0: 0}
    best = 0
    stack = [0]
    while stack:
        i = stack.pop()
        for s in range(2):
            if ck[i, s] == 1:
                depth[ci[i, s]] = depth[i] + 1
                stack.append(ci[i, s])
            else:
                best = max(best, depth[i] + 1)
    assert t.height == best


# ---------------------------------------------------------------- spatial

@pytest.mark.parametrize("fmt", ["fp32", "q16"])
@pytest.mark.parametrize("sort_queries", [True, False])
def test_spatial_within_C1(orc, fmt, sort_queries):
    pts, q = datagen.config_inputs("C1")
    r = datagen.CONFIGS["C1"]["radius"]
    t = abx.bvh_build(dev(pts), node_format=fmt)
    off, idx = abx.query_spatial(t, dev(q), radius=r, sort_queries=sort_queries)
    ex = check_spatial(orc, pts, 0, q, orc.WITHIN, host(off), host(idx), radius=r)
    assert ex <= 20


def test_spatial_within_boxes_and_radii(orc):
    pts = datagen.uniform_cube(9000, 21)
    boxes = datagen.boxes_around(pts, 22, 0.01)
    q = datagen.uniform_cube(7001, 23)
    radii = np.random.default_rng(24).uniform(-0.01, 0.05, size=7001).astype(np.float32)
    for fmt in ("fp32", "q16"):
        t = abx.bvh_build(dev(boxes), kind=1, node_format=fmt)
        off, idx = abx.query_spatial(t, dev(q), radii=dev(radii))
        check_spatial(orc, boxes, 1, q, orc.WITHIN, host(off), host(idx), radii=radii)


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("fmt", ["fp32", "q16"])
def test_spatial_intersects_exact(orc, kind, fmt):
    pts = datagen.clusters(11_000, 31)
    prims = pts if kind == 0 else datagen.boxes_around(pts, 32, 0.005)
    c = datagen.uniform_cube(6000, 33)
    h = np.float32(datagen.box_side_for_density(11_000) / 2)
    qb = np.concatenate([c - h, c + h], axis=1).astype(np.float32)
    t = abx.bvh_build(dev(prims), kind=kind, node_format=fmt)
    off, idx = abx.query_spatial(t, dev(qb), predicate="intersects")
    assert check_spatial(orc, prims, kind, qb, orc.INTERSECTS, host(off), host(idx)) == 0


def test_spatial_capacity_path(orc):
    pts, q = datagen.config_inputs("C1", n=5000, m=3000)
    t = abx.bvh_build(dev(pts))
    off, idx = abx.query_spatial(t, dev(q), radius=0.1, capacity=10)     # too small
    off2, idx2 = abx.query_spatial(t, dev(q), radius=0.1, capacity=10 ** 6)  # one pass
    o, i = host(off), host(idx)
    assert np.array_equal(o, host(off2))
    for j in range(3000):
        assert sorted(i[o[j]:o[j + 1]]) == sorted(host(idx2)[o[j]:o[j + 1]])
    check_spatial(orc, pts, 0, q, orc.WITHIN, o, i, radius=0.1)


def test_spatial_edge_cases(orc):
    q = dev(datagen.uniform_cube(100, 1))
    empty = abx.bvh_build(dev(np.zeros((0, 3), np.float32)))
    off, idx = abx.query_spatial(empty, q, radius=1.0)
    assert host(off).tolist() == [0] * 101 and idx.numel() == 0
    one = abx.bvh_build(dev(np.array([[0.5, 0.5, 0.5]], np.float32)))
    off, idx = abx.query_spatial(one, q, radius=0.3)
    check_spatial(orc, np.array([[0.5, 0.5, 0.5]], np.float32), 0, host(q), orc.WITHIN, host(off),
                  host(idx), radius=0.3)
    t = abx.bvh_build(dev(datagen.uniform_cube(1000, 2)))
    off, idx = abx.query_spatial(t, dev(np.zeros((0, 3), np.float32)), radius=1.0)
    assert host(off).tolist() == [0]
    off, idx = abx.query_spatial(t, q, radius=-1.0)
    assert host(off).tolist() == [0] * 101


# ---------------------------------------------------------------- nearest

@pytest.mark.parametrize("k", [1, 5, 10, 16, 32])
def test_nearest_C1(orc, k):
    pts, q = datagen.config_inputs("C1")
    t = abx.bvh_build(dev(pts))
    off, idx, dist = abx.query_nearest(t, dev(q), k)
    assert host(off).tolist() == list(range(0, k * len(q) + 1, k))
    check_nearest(orc, pts, 0, q, k, host(idx), host(dist))


@pytest.mark.parametrize("kind", [0, 1])
def test_nearest_q16_and_boxes(orc, kind):
    pts = datagen.clusters(10_007, 41)
    prims = pts if kind == 0 else datagen.boxes_around(pts, 42, 0.004)
    q = datagen.uniform_cube(5003, 43)
    for fmt in ("fp32", "q16"):
        t = abx.bvh_build(dev(prims), kind=kind, node_format=fmt)
        off, idx, dist = abx.query_nearest(t, dev(q), 10)
        check_nearest(orc, prims, kind, q, 10, host(idx), host(dist))


def test_nearest_edge_cases(orc):
    pts = datagen.uniform_cube(7, 1)
    q = datagen.uniform_cube(50, 2)
    t = abx.bvh_build(dev(pts))
    off, idx, dist = abx.query_nearest(t, dev(q), 12)       # k > n: all n, purged rows
    assert idx.shape == (50, 7)
    check_nearest(orc, pts, 0, q, 12, host(idx), host(dist))
    off, idx, dist = abx.query_nearest(t, dev(q), 0)
    assert idx.shape == (50, 0) and host(off).tolist() == [0] * 51
    empty = abx.bvh_build(dev(np.zeros((0, 3), np.float32)))
    off, idx, dist = abx.query_nearest(empty, dev(q), 3)
    assert idx.shape == (50, 0)
    one = abx.bvh_build(dev(pts[:1]))
    off, idx, dist = abx.query_nearest(one, dev(q), 3)
    check_nearest(orc, pts[:1], 0, q, 3, host(idx), host(dist))
    # duplicates: ties resolved by index
    dup = np.repeat(pts, 5, axis=0)
    t = abx.bvh_build(dev(dup))
    off, idx, dist = abx.query_nearest(t, dev(q), 8)
    oi, od = orc.nearest(dup, 0, q, 8)
    assert np.array_equal(host(idx), oi)


# ---------------------------------------------------------------- variants agree bitwise

def test_variants_bitwise_equal(orc):
    pts = datagen.shell(30_000, 51, 1 - 5e-3, 1 + 5e-3)
    q = datagen.uniform_cube(20_000, 52, -1.0, 1.0)
    r = float(np.float32(0.02))
    res, csr = {}, None
    for fmt, order in (("fp32", "auto"), ("q16", "build"), ("q16", "depth_first")):
        t = abx.bvh_build(dev(pts), node_format=fmt, node_order=order)
        for sq in (True, False):
            off, idx = abx.query_spatial(t, dev(q), radius=r, sort_queries=sq)
            o, i = host(off), host(idx)
            csr = csr or (o, i)
            rows = [tuple(sorted(i[o[j]:o[j + 1]].tolist())) for j in range(len(q))]
            _, ki, kd = abx.query_nearest(t, dev(q), 10, sort_queries=sq)
            res[(fmt, order, sq)] = (o.tolist(), rows, host(ki).tobytes(), host(kd).tobytes())
    first = next(iter(res.values()))
    for v in res.values():
        assert v == first
    check_spatial(orc, pts, 0, q, orc.WITHIN, csr[0], csr[1], radius=r,
                  rows=np.arange(0, 20_000, 97))


def test_stats_consistent_with_results(orc):
    pts, q = datagen.config_inputs("C1")
    r = datagen.CONFIGS["C1"]["radius"]
    for fmt in ("fp32", "q16"):
        # point trees hold every leaf's exact box in its parent node: no
        # leaf record is read
        t = abx.bvh_build(dev(pts), node_format=fmt)
        st = host(abx.query_spatial_stats(t, dev(q), radius=r))
        assert np.all(st[:, 0] >= 1) and np.all(st[:, 1] == 0)
        sn = host(abx.query_nearest_stats(t, dev(q), 10))
        assert np.all(sn[:, 0] >= 1) and np.all(sn[:, 1] == 0)
    # Q16 box trees confirm each candidate with its exact box record: every
    # emitted primitive was read at least once
    boxes = datagen.boxes_around(pts, 3, 0.002)
    t = abx.bvh_build(dev(boxes), kind=1, node_format="q16")
    st = host(abx.query_spatial_stats(t, dev(q), radius=r))
    off, _ = abx.query_spatial(t, dev(q), radius=r)
    assert np.all(st[:, 1] >= np.diff(host(off)))
    sn = host(abx.query_nearest_stats(t, dev(q), 10))
    assert np.all(sn[:, 1] >= 10)


# ---------------------------------------------------------------- cooperative nearest pass

@pytest.mark.parametrize("budget", [1, 7, 64])
@pytest.mark.parametrize("fmt", ["fp32", "q16"])
def test_nearest_cooperative_pass(orc, budget, fmt):
    # a tiny visit budget sends (almost) every query through the wavefront-
    # per-query pass; results must match the oracle and the one-lane pass
    pts = datagen.shell(20_000, 61, 1 - 5e-3, 1 + 5e-3)
    q = datagen.uniform_cube(3001, 62, -1.0, 1.0)
    t = abx.bvh_build(dev(pts), node_format=fmt)
    old = abx.set_nearest_budget(0)
    try:
        _, i1, d1 = abx.query_nearest(t, dev(q), 10)
        abx.set_nearest_budget(budget)
        for k in (1, 10, 16):
            _, ik, dk = abx.query_nearest(t, dev(q), k)
            check_nearest(orc, pts, 0, q, k, host(ik), host(dk))
            if k == 10:
                assert np.array_equal(host(ik), host(i1)) and np.array_equal(host(dk), host(d1))
    finally:
        abx.set_nearest_budget(old)


@pytest.mark.parametrize("fmt", ["fp32", "q16"])
def test_nearest_cooperative_pass_large_lists(orc, fmt):
    # the 48- and 64-key lists through the cooperative pass (budget 1), equal
    # to the one-lane walk bit for bit
    pts = datagen.shell(20_000, 63, 1 - 5e-3, 1 + 5e-3)
    q = datagen.uniform_cube(1501, 64, -1.0, 1.0)
    t = abx.bvh_build(dev(pts), node_format=fmt)
    old = abx.set_nearest_budget(0)
    try:
        for k in (40, 64):
            abx.set_nearest_budget(0)
            _, i1, d1 = abx.query_nearest(t, dev(q), k)
            abx.set_nearest_budget(1)
            _, ik, dk = abx.query_nearest(t, dev(q), k)
            assert np.array_equal(host(ik), host(i1)) and np.array_equal(host(dk), host(d1))
            check_nearest(orc, pts, 0, q, k, host(ik), host(dk), rows=np.arange(0, 1501, 7))
    finally:
        abx.set_nearest_budget(old)


def test_nearest_cooperative_boxes_and_ties(orc):
    pts = np.repeat(datagen.uniform_cube(2000, 71), 3, axis=0)     # triplicated points
    boxes = datagen.boxes_around(datagen.clusters(6000, 72), 73, 0.01)
    q = datagen.uniform_cube(999, 74)
    old = abx.set_nearest_budget(3)
    try:
        t = abx.bvh_build(dev(pts))
        _, i, d = abx.query_nearest(t, dev(q), 8)
        oi, od = orc.nearest(pts, 0, q, 8)
        assert np.array_equal(host(i), oi)
        for fmt in ("fp32", "q16"):
            t = abx.bvh_build(dev(boxes), kind=1, node_format=fmt)
            _, i, d = abx.query_nearest(t, dev(q), 10)
            check_nearest(orc, boxes, 1, q, 10, host(i), host(d))
    finally:
        abx.set_nearest_budget(old)


def test_nearest_nan_and_infinite_queries(orc):
    # a NaN coordinate adds no gap on its axis (IEEE max drops NaN; the
    # oracle's comparisons do the same); an infinite one puts everything at
    # +inf, where the tie rule picks the smallest indices
    pts = datagen.uniform_cube(5_000, 81)
    q = datagen.uniform_cube(300, 82)
    q[7] = [np.nan, 0.5, 0.5]
    q[8] = [np.inf, 0.5, 0.5]
    q[9] = [-np.inf, np.inf, 0.5]
    for fmt in ("fp32", "q16"):
        t = abx.bvh_build(dev(pts), node_format=fmt)
        _, ki, kd = abx.query_nearest(t, dev(q), 6)
        ki, kd = host(ki), host(kd)
        check_nearest(orc, pts, 0, q, 6, ki, kd, rows=[0, 7, 100])
        for r in (8, 9):
            assert ki[r].tolist() == list(range(6)) and np.all(np.isinf(kd[r]))
        off, idx = abx.query_spatial(t, dev(q), radius=0.05)
        check_spatial(orc, pts, 0, q, orc.WITHIN, host(off), host(idx), radius=0.05,
                      rows=[0, 7, 8, 9])
        cnt = np.diff(host(off))
        assert cnt[7] > 0 and cnt[8] == 0 and cnt[9] == 0


@pytest.mark.parametrize("k", [33, 48, 49, 64, 65, 100, 128])
def test_nearest_large_k(orc, k):
    # 33..64: register lists of 48 or 64 keys; 65..128: per-lane LDS max-heaps
    pts = datagen.clusters(20_000, 91)
    q = datagen.uniform_cube(2_001, 92)
    boxes = datagen.boxes_around(pts, 93, 0.003)
    for kind, prims in ((0, pts), (1, boxes)):
        for fmt in ("fp32", "q16"):
            t = abx.bvh_build(dev(prims), kind=kind, node_format=fmt)
            off, ki, kd = abx.query_nearest(t, dev(q), k)
            assert host(off)[-1] == 2_001 * k
            check_nearest(orc, prims, kind, q, k, host(ki), host(kd),
                          rows=np.arange(0, 2_001, 23))
            st = host(abx.query_nearest_stats(t, dev(q), k))
            assert np.all(st[:, 0] >= 1)


def test_nearest_large_k_edges(orc):
    pts = datagen.uniform_cube(50, 94)
    q = datagen.uniform_cube(70, 95)
    t = abx.bvh_build(dev(pts), node_format="q16")
    _, ki, kd = abx.query_nearest(t, dev(q), 100)          # k > n: rows of n
    assert host(ki).shape == (70, 50)
    check_nearest(orc, pts, 0, q, 100, host(ki), host(kd))
    one = abx.bvh_build(dev(np.array([[0.5, 0.5, 0.5]], np.float32)))
    _, ki, kd = abx.query_nearest(one, dev(q), 64)
    assert host(ki).shape == (70, 1) and np.all(host(ki) == 0)
    big = abx.bvh_build(dev(datagen.uniform_cube(500, 96)))
    with pytest.raises(abx.AbxError) as e:
        abx.query_nearest(big, dev(q), 129)
    assert e.value.status == abx.ERR_UNSUPPORTED
