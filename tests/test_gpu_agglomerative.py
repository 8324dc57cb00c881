"""GPU parity of the agglomerative (single bottom-up pass) construction: the
same binary radix tree as the Karras build and the oracle, numbered by split,
with identical boxes and identical query results.  Sizes straddle the 8192-
leaf chunk so both phases of the climb run.  Runs only on an MI355X."""
import numpy as np
import pytest
import torch

from paper_1908_11807_amd import abx, datagen
from parity import check_nearest, decode_tree

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def canon(child_kind, child_index, n, root):
    """{(first, last, split)} of every internal node, and the child boxes'
    owner map (first, last, side) -> (node, side), numbering-independent."""
    ck, ci = child_kind, child_index
    rng = {}
    order, stack = [], [root]
    while stack:                              # pre-order, then reverse
        v = stack.pop()
        order.append(v)
        for s in range(2):
            if ck[v, s] == 1:
                stack.append(ci[v, s])
    assert len(order) == n - 1, "every internal node reachable once"
    for v in reversed(order):
        ends = []
        for s in range(2):
            if ck[v, s] == 1:
                ends.append(rng[ci[v, s]])
            else:
                ends.append((ci[v, s], ci[v, s]))
        assert ends[0][1] + 1 == ends[1][0], "children cover adjacent ranges"
        rng[v] = (ends[0][0], ends[1][1], ends[0][1])
    topo = set(rng.values())
    owner = {}
    for v, (a, b, s) in rng.items():
        owner[(a, s, 0)] = (v, 0)
        owner[(s + 1, b, 1)] = (v, 1)
    return topo, owner, rng


def oracle_topology(ref, n):
    return canon(ref["child_kind"], ref["child_index"], n, 0)[0]


@pytest.mark.parametrize("n", [2, 3, 1000, 8192, 8193, 40_000])
@pytest.mark.parametrize("kind", [0, 1])
def test_same_tree_as_karras_and_oracle(orc, n, kind):
    pts = datagen.clusters(n, 700 + n)
    prims = pts if kind == 0 else datagen.boxes_around(pts, 701, 0.003)
    for fmt in ("fp32", "q16"):
        tk = abx.bvh_build(dev(prims), kind=kind, node_format=fmt)
        ta = abx.bvh_build(dev(prims), kind=kind, node_format=fmt, hierarchy="agglomerative")
        la, lk = ta.layout, tk.layout
        assert la.hierarchy == 1 and lk.hierarchy == 0 and lk.root == 0
        assert la.height == lk.height
        da, dk = decode_tree(ta), decode_tree(tk)
        assert np.array_equal(da["perm"], dk["perm"])
        topo_a, own_a, _ = canon(da["child_kind"], da["child_index"], n, la.root)
        topo_k, own_k, _ = canon(dk["child_kind"], dk["child_index"], n, 0)
        assert topo_a == topo_k
        if fmt == "fp32" and n <= 8193:
            assert topo_a == oracle_topology(orc.build(prims, kind, 21), n)
        # every child box equal, matched by the child's leaf range
        for key, (va, sa) in own_a.items():
            vk, sk = own_k[key]
            if fmt == "fp32":
                ba = da["boxes_l"][va] if sa == 0 else da["boxes_r"][va]
                bk = dk["boxes_l"][vk] if sk == 0 else dk["boxes_r"][vk]
            else:
                ba = da["q_l"][va] if sa == 0 else da["q_r"][va]
                bk = dk["q_l"][vk] if sk == 0 else dk["q_r"][vk]
            assert np.array_equal(ba, bk), key
        if fmt == "q16":
            np.testing.assert_array_equal(da["leaf_boxes"], dk["leaf_boxes"])


def test_duplicates_and_query_results_identical(orc):
    rng = np.random.default_rng(9)
    pts = rng.integers(0, 6, size=(30_000, 3)).astype(np.float32)    # heavy duplicates
    q = datagen.uniform_cube(5_001, 10, 0.0, 5.0)
    for fmt in ("fp32", "q16"):
        tk = abx.bvh_build(dev(pts), node_format=fmt)
        ta = abx.bvh_build(dev(pts), node_format=fmt, hierarchy="agglomerative")
        da, dk = decode_tree(ta), decode_tree(tk)
        assert canon(da["child_kind"], da["child_index"], 30_000, ta.layout.root)[0] == \
            canon(dk["child_kind"], dk["child_index"], 30_000, 0)[0]
        ok, ik = abx.query_spatial(tk, dev(q), radius=0.9)
        oa, ia = abx.query_spatial(ta, dev(q), radius=0.9)
        assert np.array_equal(host(ok), host(oa)) and np.array_equal(host(ik), host(ia))
        _, nk, dk_ = abx.query_nearest(tk, dev(q), 16)
        _, na, da_ = abx.query_nearest(ta, dev(q), 16)
        assert np.array_equal(host(nk), host(na)) and np.array_equal(host(dk_), host(da_))
    check_nearest(orc, pts, 0, q[:300], 16, host(na)[:300], host(da_)[:300])


def test_shell_nearest_and_one_point():
    pts = datagen.shell(100_000, 11)
    q = datagen.uniform_cube(20_000, 12, -1.0, 1.0)
    tk = abx.bvh_build(dev(pts), node_format="q16")
    ta = abx.bvh_build(dev(pts), node_format="q16", hierarchy="agglomerative")
    _, nk, dk = abx.query_nearest(tk, dev(q), 10)
    _, na, da = abx.query_nearest(ta, dev(q), 10)
    assert np.array_equal(host(nk), host(na)) and np.array_equal(host(dk), host(da))
    one = abx.bvh_build(dev(np.array([[0.25, 0.5, 0.75]], np.float32)), hierarchy="agglomerative")
    _, i1, d1 = abx.query_nearest(one, dev(np.array([[0.25, 0.5, 0.5]], np.float32)), 3)
    assert host(i1).tolist() == [[0]] and abs(float(host(d1)[0, 0]) - 0.25) < 1e-7


def _sorted_rows(a):
    a = np.ascontiguousarray(a)
    return a[np.lexsort(a.T[::-1])]


@pytest.mark.parametrize("n", [524_288, 524_289])
def test_group_edges_same_boxes(n):
    pts = datagen.clusters(n, 81)
    tk = abx.bvh_build(dev(pts), node_format="fp32")
    ta = abx.bvh_build(dev(pts), node_format="fp32", hierarchy="agglomerative")
    assert ta.layout.height == tk.layout.height
    da, dk = decode_tree(ta), decode_tree(tk)
    rows_a = _sorted_rows(np.concatenate([da["boxes_l"], da["boxes_r"]]))
    rows_k = _sorted_rows(np.concatenate([dk["boxes_l"], dk["boxes_r"]]))
    assert np.array_equal(rows_a, rows_k)


@pytest.mark.parametrize("fmt", ["fp32", "q16"])
def test_large_tree_all_build_phases(orc, fmt):
    # 1.3e6 leaves: 159 chunks in three groups of 64 (the last ragged), so the
    # chunk, group and top passes of both hierarchy builds all run.  The two
    # builds make the same binary radix tree under different node numbering:
    # the multisets of child boxes are equal, and so are query results.
    n = 1_300_000
    pts = datagen.shell(n, 79, 0.99, 1.01)
    tk = abx.bvh_build(dev(pts), node_format=fmt)
    ta = abx.bvh_build(dev(pts), node_format=fmt, hierarchy="agglomerative")
    assert ta.layout.height == tk.layout.height
    da, dk = decode_tree(ta), decode_tree(tk)
    assert np.array_equal(da["perm"], dk["perm"])
    keys = ("boxes_l", "boxes_r") if fmt == "fp32" else ("q_l", "q_r")
    for d in (da, dk):
        assert np.sum(d["child_kind"] == 0) == n   # every leaf referenced once
    rows_a = _sorted_rows(np.concatenate([da[keys[0]], da[keys[1]]]))
    rows_k = _sorted_rows(np.concatenate([dk[keys[0]], dk[keys[1]]]))
    assert np.array_equal(rows_a, rows_k)
    q = datagen.uniform_cube(100_000, 80, -1.0, 1.0)
    _, ia, da_ = abx.query_nearest(ta, dev(q), 10)
    _, ik, dk_ = abx.query_nearest(tk, dev(q), 10)
    assert torch.equal(ia, ik) and torch.equal(da_, dk_)
    check_nearest(orc, pts, 0, q[::997], 10, ia.cpu().numpy()[::997], da_.cpu().numpy()[::997])
