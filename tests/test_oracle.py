"""Pins for the CPU oracle, independent of the oracle's own code.

Every check here compares the oracle with something other than itself:
values printed in the paper (Fig. 1 of section 2), values worked by hand
from the definitions of section 2.1, textbook closed forms (lattice-point
counts), an independent library (scipy's k-d tree), an independent
construction (a binary trie), or exact invariants of the definitions of
section 2.2.  None of these tests touches a GPU.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

from conftest import golden_path
from paper_1908_11807_amd import datagen

UNIT = np.array([0, 0, 0, 1, 1, 1], np.float32)


def _read_rows(name):
    rows = []
    with open(golden_path(name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(line.split())
    return rows


# ----------------------------------------------------------------- Morton codes

def test_morton_handworked(orc):
    rows = _read_rows("morton_handworked.txt")
    pts = np.array([[float(r[0]), float(r[1]), float(r[2])] for r in rows], np.float32)
    c10 = orc.morton(pts, orc.POINTS, UNIT, 10)
    c21 = orc.morton(pts, orc.POINTS, UNIT, 21)
    assert [int(c) for c in c10] == [int(r[3], 16) for r in rows]
    assert [int(c) for c in c21] == [int(r[4], 16) for r in rows]


def _deinterleave(code, bits):
    q = [0, 0, 0]
    for b in range(bits):
        for a in range(3):
            q[a] |= ((code >> (3 * b + (2 - a))) & 1) << b
    return q


@pytest.mark.parametrize("bits", [10, 21])
def test_morton_dyadic_grid_roundtrip(orc, bits):
    # points i / 2^bits are exact in float32 and normalise exactly in the unit
    # scene box, so the quantised coordinate must be i itself
    rng = np.random.default_rng(7)
    q = rng.integers(0, 2 ** bits, size=(300, 3))
    pts = (q / float(2 ** bits)).astype(np.float32)
    assert np.all(pts.astype(np.float64) * 2 ** bits == q)
    codes = orc.morton(pts, orc.POINTS, UNIT, bits)
    for c, qq in zip(codes, q):
        assert _deinterleave(int(c), bits) == list(qq)
        assert int(c) < 2 ** (3 * bits)


def test_morton_box_centroid_and_degenerate_axis(orc):
    # a box's code is its centroid's code; an axis of zero scene extent
    # contributes zero bits
    p = np.array([[0.25, 0.5, 0.0], [0.75, 0.125, 0.0]], np.float32)
    h = np.float32(0.0625)
    boxes = np.concatenate([p - h, p + h], axis=1).astype(np.float32)
    scene = np.array([0, 0, 0, 1, 1, 0], np.float32)
    cb = orc.morton(boxes, orc.BOXES, scene, 10)
    cp = orc.morton(p, orc.POINTS, scene, 10)
    assert list(cb) == list(cp)
    for c in cp:
        assert _deinterleave(int(c), 10)[2] == 0
    assert int(cp[0]) == int(orc.morton(np.array([[0.25, 0.5, 0.0]], np.float32), 0, UNIT, 10)[0])


def test_morton_clamps_outside_scene(orc):
    pts = np.array([[-1, -1, -1], [2, 2, 2]], np.float32)
    c = orc.morton(pts, orc.POINTS, UNIT, 10)
    assert list(map(int, c)) == [0, 2 ** 30 - 1]


# ------------------------------------------------------- Fig. 1 of section 2

def _fig1():
    leaves, nodes = {}, {}
    for r in _read_rows("fig1_bvh.txt"):
        box = np.array([float(r[2]), float(r[3]), 0.0, float(r[4]), float(r[5]), 0.0], np.float32)
        if r[0] == "leaf":
            leaves[int(r[1])] = box
        else:
            nodes[int(r[1])] = (box, (int(r[7]), int(r[8])))
    return leaves, nodes


def _oracle_leafsets(t):
    """leaf set (original indices) of every internal node, and of its two children"""
    perm = t["perm"]
    out = {}
    for i, (f, l) in enumerate(t["range"]):
        kids = []
        for s in range(2):
            if t["child_kind"][i, s] == 0:
                kids.append(frozenset([int(perm[t["child_index"][i, s]])]))
            else:
                cf, cl = t["range"][t["child_index"][i, s]]
                kids.append(frozenset(int(x) for x in perm[cf:cl + 1]))
        out[frozenset(int(x) for x in perm[f:l + 1])] = (i, frozenset(kids))
    return out


@pytest.mark.parametrize("bits", [10, 21])
def test_fig1_topology_and_boxes(orc, bits):
    leaves, nodes = _fig1()
    prims = np.stack([leaves[i] for i in range(8)])
    t = orc.build(prims, orc.BOXES, bits)
    assert t["child_kind"].shape == (7, 2)          # n - 1 internal nodes

    # leaf sets of the figure's internal nodes, from their printed children
    def fig_set(j):
        return frozenset([j]) if j < 8 else frozenset().union(*[fig_set(c) for c in nodes[j][1]])

    fig = {fig_set(j): frozenset(fig_set(c) for c in nodes[j][1]) for j in nodes}
    ours = _oracle_leafsets(t)
    assert set(fig) == set(ours)
    for s, kids in fig.items():
        i, okids = ours[s]
        assert okids == kids
        # internal box equals the figure's box exactly
        fig_box = [nodes[j][0] for j in nodes if fig_set(j) == s][0]
        np.testing.assert_array_equal(t["boxes"][i], fig_box)
    np.testing.assert_array_equal(t["boxes"][0], t["scene"])     # root = scene box
    np.testing.assert_array_equal(t["scene"], nodes[14][0])


def test_fig1_y_major_interleave_does_not_match(orc):
    # x must be the most significant coordinate: swapping x and y (a y-major
    # interleave) yields a tree that is not the figure's
    leaves, nodes = _fig1()
    prims = np.stack([leaves[i] for i in range(8)])
    swapped = prims[:, [1, 0, 2, 4, 3, 5]].copy()
    t = orc.build(swapped, orc.BOXES, 10)
    fig_sets = {frozenset([1, 5]), frozenset([4, 6]), frozenset([0, 4, 6]), frozenset([2, 7]),
                frozenset([1, 3, 5]), frozenset([0, 2, 4, 6, 7])}
    assert set(_oracle_leafsets(t)) - {frozenset(range(8))} != fig_sets


# ----------------------------------------------------- hierarchy = radix tree

def _trie_structure(sorted_codes, keybits):
    """Independent construction: insert every index-augmented key into a
    binary trie bit by bit, then read off the branching nodes."""
    n = len(sorted_codes)
    strings = [format(int(c), "0%db" % keybits) + format(p, "032b") for p, c in enumerate(sorted_codes)]
    root = {}
    for p, s in enumerate(strings):
        node = root
        for ch in s:
            node = node.setdefault(ch, {})
        node["leaf"] = p

    def collect(node):
        if "leaf" in node:
            return frozenset([node["leaf"]]), []
        kids = [collect(node[ch]) for ch in "01" if ch in node]
        sets = [k[0] for k in kids]
        branches = sum((k[1] for k in kids), [])
        mine = frozenset().union(*sets)
        if len(kids) == 2:
            branches.append((mine, frozenset(sets)))
        return mine, branches

    _, br = collect(root)
    return {s: kids for s, kids in br}


@pytest.mark.parametrize("seed", range(6))
def test_hierarchy_equals_binary_radix_trie(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 40))
    keybits = [30, 63][seed % 2]
    # few distinct codes so that duplicates (index tie-breaks) occur
    codes = np.sort(rng.integers(0, 2 ** min(keybits, 12), size=n).astype(np.uint64)
                    << np.uint64(keybits - min(keybits, 12)))
    ck, ci, rg = orc.hierarchy(codes, keybits)
    trie = _trie_structure(codes, keybits)
    ours = {}
    for i, (f, l) in enumerate(rg):
        kids = []
        for s in range(2):
            if ck[i, s] == 0:
                kids.append(frozenset([int(ci[i, s])]))
            else:
                cf, cl = rg[ci[i, s]]
                kids.append(frozenset(range(cf, cl + 1)))
        ours[frozenset(range(f, l + 1))] = frozenset(kids)
        assert i in (f, l) or i == 0                # Karras numbering: a range end
    assert rg[0].tolist() == [0, n - 1]
    assert ours == trie


def test_hierarchy_invariants_random(orc):
    pts = datagen.uniform_cube(5000, 11)
    t = orc.build(pts, orc.POINTS, 21)
    n = 5000
    ck, ci = t["child_kind"], t["child_index"]
    assert ck.shape == (n - 1, 2)
    leaves = ci[ck == 0]
    inter = ci[ck == 1]
    # every leaf reached exactly once, every internal node but the root once
    assert sorted(leaves.tolist()) == list(range(n))
    assert sorted(inter.tolist()) == list(range(1, n - 1))


def test_refit_is_union_over_ranges(orc):
    pts = datagen.uniform_cube(3000, 12)
    t = orc.build(pts, orc.POINTS, 21)
    sp = pts[t["perm"]]
    for i, (f, l) in enumerate(t["range"]):
        seg = sp[f:l + 1]
        np.testing.assert_array_equal(t["boxes"][i, :3], seg.min(axis=0))
        np.testing.assert_array_equal(t["boxes"][i, 3:], seg.max(axis=0))
    np.testing.assert_array_equal(t["boxes"][0], t["scene"])
    np.testing.assert_array_equal(t["scene"][:3], pts.min(axis=0))


def test_scene_box_flags_inverted_box(orc):
    b = np.array([[0, 0, 0, 1, 1, 1], [0, 0, 0, 1, 1, 1]], np.float32)
    assert not orc.scene_box(b, orc.BOXES)[1]
    b[1, 4] = -0.5                      # hi.y < lo.y
    assert orc.scene_box(b, orc.BOXES)[1]


def test_scene_box_flags_nan_and_inf(orc):
    p = datagen.uniform_cube(10, 1)
    assert not orc.scene_box(p)[1]
    for bad in (np.nan, np.inf, -np.inf):
        q = p.copy()
        q[3, 1] = bad
        assert orc.scene_box(q)[1]


# --------------------------------------------------------- spatial: within

def _lattice(h=4):
    return np.array(list(itertools.product(range(-h, h + 1), repeat=3)), np.float32)


def test_within_lattice_ball_counts(orc):
    pts = _lattice()
    for s, count in ((int(a), int(b)) for a, b in _read_rows("lattice_ball_counts.txt")):
        r = math.isqrt(s) if math.isqrt(s) ** 2 == s else math.sqrt(s) + 1e-3
        off, idx = orc.spatial(pts, orc.POINTS, np.zeros((1, 3), np.float32), orc.WITHIN, radius=r)
        assert off[1] == count, (s, off[1], count)


def test_within_closed_ball_boundary(orc):
    # a point at exactly distance r is inside (reading: closed ball)
    pts = np.array([[3, 4, 0], [0, 0, 5.0000005]], np.float32)
    off, idx = orc.spatial(pts, orc.POINTS, np.zeros((1, 3), np.float32), orc.WITHIN, radius=5.0)
    assert idx.tolist() == [0]


def test_within_matches_scipy_kdtree(orc):
    pts = datagen.uniform_cube(3000, 21)
    q = datagen.uniform_cube(400, 22)
    r = 0.08
    off, idx = orc.spatial(pts, orc.POINTS, q, orc.WITHIN, radius=r)
    tree = cKDTree(pts.astype(np.float64))
    ref = tree.query_ball_point(q.astype(np.float64), float(np.float32(r)))
    for j in range(len(q)):
        got = set(idx[off[j]:off[j + 1]].tolist())
        d = orc.distances(pts, orc.POINTS, q[j])
        band = set(np.nonzero(np.abs(d - np.float32(r)) <= 1e-12)[0].tolist())
        assert got - band == set(ref[j]) - band


def test_within_per_query_radii_and_negative(orc):
    pts = datagen.uniform_cube(500, 31)
    q = datagen.uniform_cube(50, 32)
    radii = np.linspace(-0.1, 0.3, 50).astype(np.float32)
    off, idx = orc.spatial(pts, orc.POINTS, q, orc.WITHIN, radii=radii)
    for j in range(50):
        off1, idx1 = orc.spatial(pts, orc.POINTS, q[j:j + 1], orc.WITHIN, radius=radii[j])
        assert idx[off[j]:off[j + 1]].tolist() == idx1.tolist()
        if radii[j] < 0:
            assert off[j + 1] == off[j]


def test_within_self_join_symmetric_and_monotone(orc):
    pts = datagen.uniform_cube(1500, 41)
    r = 0.06
    off, idx = orc.spatial(pts, orc.POINTS, pts, orc.WITHIN, radius=r)
    pairs = {(j, int(i)) for j in range(len(pts)) for i in idx[off[j]:off[j + 1]]}
    assert all((i, j) in pairs for j, i in pairs)
    assert all((j, j) in pairs for j in range(len(pts)))
    off2, idx2 = orc.spatial(pts, orc.POINTS, pts, orc.WITHIN, radius=r * 1.3)
    for j in range(len(pts)):
        assert set(idx[off[j]:off[j + 1]]) <= set(idx2[off2[j]:off2[j + 1]])


def test_radius_rule_expected_count_unit_cube(orc):
    # section 3: r such that a filled cube holds k = 10 neighbours on average.
    # In the unit cube the boundary cuts the mean to 10 (1 - 9r/8): the
    # fraction of the ball outside a face at depth x is averaged over x.
    c = datagen.CONFIGS["C1"]
    assert abs(c["radius"] - 0.06203505) < 1e-7
    pts, q = datagen.config_inputs("C1")
    off, _ = orc.spatial(pts, orc.POINTS, q, orc.WITHIN, radius=c["radius"])
    mean = off[-1] / len(q)
    assert abs(mean - 10 * (1 - 9 * c["radius"] / 8)) < 0.15, mean


def test_radius_rule_paper_filled_case(orc):
    # the paper's filled case (filled sphere queries in a filled cube of
    # density 1/8, r = (6k/pi)^(1/3)) averages 10 neighbours (section 3,
    # spatial search rates); weak pin: the size is not stated in the paper
    p = 40_000
    r = datagen.radius_for_density(p, 10, volume=(2 * p ** (1 / 3)) ** 3)
    assert abs(r - (60 / math.pi) ** (1 / 3)) < 1e-9
    src = datagen.paper_filled_cube(p, 1)
    q = datagen.paper_filled_sphere(4000, 2)
    a = p ** (1 / 3)
    inner = q[np.linalg.norm(q, axis=1) < a - r]     # balls fully inside the cube
    off, _ = orc.spatial(src, orc.POINTS, inner, orc.WITHIN, radius=r)
    assert abs(off[-1] / len(inner) - 10.0) < 0.3


def test_shell_radius_rule(orc):
    # a query on the shell's mid-surface sees (n/4)(r^2 - t^2/12) points
    n, t = 200_000, 1e-2
    r = datagen.radius_for_shell(n, t, 10)
    pts = datagen.shell(n, 5, 1 - t / 2, 1 + t / 2)
    d = np.random.default_rng(6).standard_normal((3000, 3))
    q = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    off, _ = orc.spatial(pts, orc.POINTS, q, orc.WITHIN, radius=r)
    assert abs(off[-1] / len(q) - 10.0) < 0.35


# ------------------------------------------------------ box primitives / boxes

def test_point_to_box_distance_handworked(orc):
    box = np.array([[0, 0, 0, 1, 1, 1]], np.float32)
    cases = [((0.5, 0.5, 0.5), 0.0), ((2, 0.5, 0.5), 1.0), ((2, 2, 2), math.sqrt(3)),
             ((-1, 0.5, 3), math.sqrt(5)), ((1, 1, 1), 0.0), ((0.5, -0.25, 0.5), 0.25)]
    for q, d in cases:
        got = orc.distances(box, orc.BOXES, np.array(q, np.float32))[0]
        assert abs(got - d) <= 1e-15 * max(1.0, d)


def test_degenerate_boxes_equal_points(orc):
    pts = datagen.uniform_cube(800, 51)
    boxes = np.concatenate([pts, pts], axis=1)
    q = datagen.uniform_cube(100, 52)
    a = orc.spatial(pts, orc.POINTS, q, orc.WITHIN, radius=0.1)
    b = orc.spatial(boxes, orc.BOXES, q, orc.WITHIN, radius=0.1)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    ka = orc.nearest(pts, orc.POINTS, q, 7)
    kb = orc.nearest(boxes, orc.BOXES, q, 7)
    assert np.array_equal(ka[0], kb[0]) and np.array_equal(ka[1], kb[1])


def test_intersects_handworked_closed_intervals(orc):
    prims = np.array([[0, 0, 0, 1, 1, 1], [2, 2, 2, 3, 3, 3], [1, 0, 0, 2, 1, 1]], np.float32)
    qb = np.array([[1, 1, 1, 2, 2, 2],                     # touches all three at faces/corners
                   [1.0000001, 0, 0, 1.9999999, 1, 1],     # strictly between 0 and 1, inside 2
                   [5, 5, 5, 6, 6, 6]], np.float32)        # touches none
    off, idx = orc.spatial(prims, orc.BOXES, qb, orc.INTERSECTS)
    rows = [sorted(idx[off[j]:off[j + 1]].tolist()) for j in range(3)]
    assert rows == [[0, 1, 2], [2], []]


def test_intersects_points_matches_chebyshev_kdtree(orc):
    pts = datagen.uniform_cube(3000, 61)
    c = datagen.uniform_cube(300, 62)
    h = np.float32(0.05)
    qb = np.concatenate([c - h, c + h], axis=1).astype(np.float32)
    off, idx = orc.spatial(pts, orc.POINTS, qb, orc.INTERSECTS)
    lo, hi = qb[:, :3].astype(np.float64), qb[:, 3:].astype(np.float64)
    cen, half = (lo + hi) / 2, (hi - lo) / 2               # exact in float64
    tree = cKDTree(pts.astype(np.float64))
    for j in range(len(c)):
        # a cube box is a Chebyshev ball; its half-widths agree to rounding
        ref = set(tree.query_ball_point(cen[j], half[j].max(), p=np.inf))
        ref = {i for i in ref if np.all(pts[i] >= qb[j, :3]) and np.all(pts[i] <= qb[j, 3:])}
        assert set(idx[off[j]:off[j + 1]].tolist()) == ref


# ------------------------------------------------------------------ nearest

def test_nearest_matches_scipy_kdtree(orc):
    pts = datagen.uniform_cube(4000, 71)
    q = datagen.uniform_cube(300, 72)
    k = 10
    idx, dist = orc.nearest(pts, orc.POINTS, q, k)
    dref, iref = cKDTree(pts.astype(np.float64)).query(q.astype(np.float64), k)
    np.testing.assert_allclose(dist, dref, rtol=1e-12, atol=0)
    assert np.array_equal(np.sort(idx, axis=1), np.sort(iref, axis=1))


def test_nearest_lattice_ties_by_index(orc):
    pts = _lattice(2)
    idx, dist = orc.nearest(pts, orc.POINTS, np.zeros((1, 3), np.float32), 7)
    origin = int(np.nonzero(np.all(pts == 0, axis=1))[0][0])
    unit = np.nonzero(np.abs(pts).sum(axis=1) == 1)[0]
    assert idx[0, 0] == origin and dist[0, 0] == 0
    assert idx[0, 1:].tolist() == sorted(unit.tolist())
    assert np.all(dist[0, 1:] == 1.0)
    # the 8th..19th nearest are the 12 points at sqrt(2), again by index
    idx2, dist2 = orc.nearest(pts, orc.POINTS, np.zeros((1, 3), np.float32), 19)
    ring = np.nonzero((pts ** 2).sum(axis=1) == 2)[0]
    assert idx2[0, 7:].tolist() == sorted(ring.tolist())


def test_nearest_invariants(orc):
    pts = datagen.clusters(3000, 81)
    q = datagen.uniform_cube(200, 82)
    i10, d10 = orc.nearest(pts, orc.POINTS, q, 10)
    i11, d11 = orc.nearest(pts, orc.POINTS, q, 11)
    assert np.all(np.diff(d10, axis=1) >= 0)                  # ascending
    assert np.array_equal(i11[:, :10], i10)                   # prefix property
    for j in range(len(q)):                                   # kNN inside within(q, d_k)
        off, idx = orc.spatial(pts, orc.POINTS, q[j:j + 1], orc.WITHIN, radius=np.nextafter(
            np.float32(d10[j, -1]), np.float32(np.inf)))
        assert set(i10[j].tolist()) <= set(idx.tolist())
        assert len(set(i10[j].tolist())) == 10


def test_nearest_degenerate_k_and_n(orc):
    pts = datagen.uniform_cube(5, 91)
    q = datagen.uniform_cube(3, 92)
    i, d = orc.nearest(pts, orc.POINTS, q, 8)                 # k > n: all n
    assert i.shape == (3, 5) and all(sorted(r) == list(range(5)) for r in i.tolist())
    i, d = orc.nearest(pts, orc.POINTS, q, 0)
    assert i.shape == (3, 0)
    i, d = orc.nearest(np.zeros((0, 3), np.float32), orc.POINTS, q, 4)
    assert i.shape == (3, 0)
    off, idx = orc.spatial(np.zeros((0, 3), np.float32), orc.POINTS, q, orc.WITHIN, radius=1.0)
    assert off.tolist() == [0, 0, 0, 0]
    one = orc.build(pts[:1], orc.POINTS, 21)                  # n = 1: no internal node
    assert one["child_kind"].shape == (0, 2) and one["perm"].tolist() == [0]


def test_paper_generators_geometry():
    # section 3 data sets: a = p^(1/3), Omega = [-a, a]^3
    p = 6_001
    a = p ** (1 / 3)
    fc = datagen.paper_filled_cube(p, 11).astype(np.float64)
    assert fc.shape == (p, 3) and np.all(np.abs(fc) <= a)
    hc = datagen.paper_hollow_cube(p, 12).astype(np.float64)
    # point i on face i mod 6: axis (i mod 6) // 2, side -a for even faces
    face = np.arange(p) % 6
    on = hc[np.arange(p), face // 2]
    np.testing.assert_allclose(on, np.where(face % 2 == 0, -a, a), rtol=1e-6)
    assert np.all(np.abs(hc) <= a * (1 + 1e-6))
    fs = datagen.paper_filled_sphere(p, 13).astype(np.float64)
    assert np.all(np.linalg.norm(fs, axis=1) <= a * (1 + 1e-6))
    hs = datagen.paper_hollow_sphere(p, 14).astype(np.float64)
    np.testing.assert_allclose(np.linalg.norm(hs, axis=1), a, rtol=1e-5)
    # the projection of a cube-uniform cloud is not uniform on the sphere:
    # directions near the cube's corners are over-represented
    d = np.abs(hs) / a
    corner = np.mean(np.min(d, axis=1) > 0.5)
    assert corner > 0.05
