"""Depth-first node order (CPU): the identity the build uses to renumber a
Karras tree -- preorder index = first leaf of the node's range + number of
ancestors whose left subtree holds it, summed by pointer jumping -- against a
plain depth-first walk of the oracle's tree, and the test helper that maps a
depth-first numbered tree back to the Karras numbering."""
import numpy as np
import pytest

import oracle
from paper_1908_11807_amd import datagen
from parity import _karras_numbering


def _dfs_order(ck, ci):
    ni = ck.shape[0]
    pre = np.full(ni, -1, np.int64)
    stack, k = [0], 0
    while stack:
        x = stack.pop()
        pre[x] = k
        k += 1
        for s in (1, 0):
            if ck[x, s] == 1:
                stack.append(ci[x, s])
    return pre


def _trees():
    for n, gen in ((2, datagen.uniform_cube), (3, datagen.uniform_cube), (17, datagen.uniform_cube),
                   (4097, datagen.clusters), (60_000, lambda n, s: datagen.shell(n, s, 0.99, 1.01))):
        p = gen(n, 5)
        yield n, oracle.build(p, oracle.POINTS, 21)


@pytest.mark.parametrize("case", range(5))
def test_preorder_identity(case):
    n, r = list(_trees())[case]
    ck, ci = r["child_kind"], r["child_index"]
    ni = n - 1
    parent = np.full(ni, -1, np.int64)
    side = np.zeros(ni, np.int64)
    for s in (0, 1):
        m = ck[:, s] == 1
        parent[ci[m, s]] = np.nonzero(m)[0]
        side[ci[m, s]] = s
    # first leaf of each node's range, by walking left
    lo = np.empty(ni, np.int64)
    for x in range(ni):
        y = x
        while ck[y, 0] == 1:
            y = ci[y, 0]
        lo[x] = ci[y, 0]
    val = ((parent >= 0) & (side == 0)).astype(np.int64)
    anc = parent.copy()
    for _ in range(7):
        has = anc >= 0
        v2, a2 = val.copy(), anc.copy()
        v2[has] = val[has] + val[anc[has]]
        a2[has] = anc[anc[has]]
        val, anc = v2, a2
    assert np.all(anc < 0)
    assert np.array_equal(lo + val, _dfs_order(ck, ci))


@pytest.mark.parametrize("case", range(5))
def test_karras_numbering_roundtrip(case):
    n, r = list(_trees())[case]
    ck, ci = r["child_kind"], r["child_index"]
    ni = n - 1
    perm = r["perm"]
    # Karras-numbered references: internal r >= 0, leaf ~primitive
    refs = np.where(ck == 1, ci, ~perm[np.clip(ci, 0, n - 1)])
    rows = np.arange(ni * 32, dtype=np.int64).reshape(ni, 32) % 251  # payload
    pre = _dfs_order(ck, ci)
    d_refs = np.where(refs >= 0, pre[np.clip(refs, 0, ni - 1)], refs)
    d_rows = np.empty_like(rows)
    d_rows[pre] = rows
    d_refs2 = np.empty_like(d_refs)
    d_refs2[pre] = d_refs
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    back_rows, back_refs = _karras_numbering(d_rows, d_refs2, n, inv)
    assert np.array_equal(back_rows, rows)
    assert np.array_equal(back_refs, refs)


@pytest.mark.parametrize("case", range(5))
def test_collapsed_wide_tree_structure(case):
    """The expected 4-wide tree (the binary tree collapsed at even depths)
    the GPU tree is compared with: every primitive appears once as a leaf
    child, every node but the root is referenced once, nodes hold 2 to 4
    children, the count is within the bound the build allocates for, and a
    node's slots cover exactly the leaves of its binary node."""
    from parity import EMPTY_REF, expected_wide
    n, r = list(_trees())[case]
    p = None
    for nn, gen in ((2, datagen.uniform_cube), (3, datagen.uniform_cube), (17, datagen.uniform_cube),
                    (4097, datagen.clusters), (60_000, lambda n, s: datagen.shell(n, s, 0.99, 1.01))):
        if nn == n:
            p = gen(n, 5)
    refs, box = expected_wide(r, p, 0, n)
    W = refs.shape[0]
    ni = n - 1
    assert 1 <= W <= (2 * ni + 1) // 3 + 1
    used = refs != EMPTY_REF
    assert np.all(used.sum(axis=1) >= 2)
    # unused slots come last
    assert np.all(np.diff(used.astype(np.int8), axis=1) <= 0)
    leaves = np.sort(~refs[used & (refs < 0)])
    assert np.array_equal(leaves, np.arange(n))
    nodes = np.sort(refs[used & (refs >= 0)])
    assert np.array_equal(nodes, np.arange(1, W))
    # depth-first numbering: each node's first internal child follows it,
    # and every child comes after its parent
    for w in range(W):
        kids = refs[w][used[w] & (refs[w] >= 0)]
        assert np.all(kids > w)
        if kids.size:
            assert kids[0] == w + 1
    # the boxes of the root's slots cover the scene box exactly
    lo = np.nanmin(box[0][used[0], :3], axis=0)
    hi = np.nanmax(box[0][used[0], 3:], axis=0)
    np.testing.assert_array_equal(np.concatenate([lo, hi]), r["scene"])
