"""Comparison rules between the HIP path and the CPU oracle.

Spatial (within): per query, the GPU index set equals the oracle's except
for pairs whose double-precision distance lies within 1e-6 relative of the
radius; those are exempt and counted.  Box intersection: exactly equal.

Nearest: row length min(k, n); GPU indices distinct and valid; the sorted
double-precision distances of the GPU's indices match the oracle's, element
by element, within 1e-6 relative; index sets equal except indices whose
distance is within 1e-6 relative of the oracle's k-th distance (exempt and
counted); each GPU float distance is within 1e-6 relative of the recomputed
double distance.
"""
import numpy as np

REL = 1e-6


def _rel_close(a, b, rel=REL):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b) <= rel * np.maximum(np.abs(a), np.abs(b))


def check_spatial(orc, prims, kind, queries, pred, gpu_off, gpu_idx, radius=0.0, radii=None,
                  rows=None):
    """Compare GPU CSR rows (all, or the sampled `rows`) with the oracle.
    Returns the number of exempt boundary pairs."""
    gpu_off = np.asarray(gpu_off, np.int64)
    gpu_idx = np.asarray(gpu_idx, np.int64)
    qw = 3 if pred == orc.WITHIN else 6
    q = np.asarray(queries, np.float32).reshape(-1, qw)
    m = q.shape[0]
    assert gpu_off.shape == (m + 1,)
    assert gpu_off[0] == 0 and np.all(np.diff(gpu_off) >= 0) and gpu_off[-1] == gpu_idx.shape[0]
    sel = np.arange(m) if rows is None else np.asarray(rows)
    rr = None if radii is None else np.asarray(radii, np.float32)[sel]
    off, idx = orc.spatial(prims, kind, q[sel], pred, radius=radius, radii=rr)
    exempt = 0
    n = np.asarray(prims).reshape(-1, 3 if kind == orc.POINTS else 6).shape[0]
    for t, j in enumerate(sel):
        g = gpu_idx[gpu_off[j]:gpu_off[j + 1]]
        assert np.all((g >= 0) & (g < n)), f"row {j}: index out of range"
        gs = set(g.tolist())
        assert len(gs) == len(g), f"row {j}: duplicate indices"
        os_ = set(idx[off[t]:off[t + 1]].tolist())
        if gs == os_:
            continue
        assert pred == orc.WITHIN, f"row {j}: box-intersection sets differ"
        r = float(np.float32(radius if radii is None else rr[t]))
        diff = np.array(sorted(gs ^ os_), np.int64)
        d = orc.distances(prims, kind, q[j], diff)
        bad = diff[~(np.abs(d - r) <= REL * r)]
        assert bad.size == 0, f"row {j}: {bad.size} non-boundary mismatches, e.g. {bad[:5]}"
        exempt += diff.size
    return exempt


def check_nearest(orc, prims, kind, queries, k, gpu_idx, gpu_dist, rows=None):
    """Returns the number of exempt tie indices."""
    q = np.asarray(queries, np.float32).reshape(-1, 3)
    n = np.asarray(prims).reshape(-1, 3 if kind == orc.POINTS else 6).shape[0]
    kk = min(k, n)
    gpu_idx = np.asarray(gpu_idx, np.int64)
    gpu_dist = np.asarray(gpu_dist, np.float64)
    m = q.shape[0]
    assert gpu_idx.shape == (m, kk) and gpu_dist.shape == (m, kk)
    sel = np.arange(m) if rows is None else np.asarray(rows)
    oi, od = orc.nearest(prims, kind, q[sel], k)
    exempt = 0
    for t, j in enumerate(sel):
        g = gpu_idx[j]
        assert np.all((g >= 0) & (g < n)), f"row {j}: invalid index"
        assert len(set(g.tolist())) == kk, f"row {j}: duplicate index"
        d64 = orc.distances(prims, kind, q[j], g)
        # rule 5: reported float distance vs recomputed double distance
        assert np.all(_rel_close(gpu_dist[j], d64) | ((gpu_dist[j] == 0) & (d64 == 0))), \
            f"row {j}: reported distance off"
        # rule 3: sorted distances match the oracle's element by element
        ds = np.sort(d64)
        assert np.all(_rel_close(ds, od[t]) | ((ds == 0) & (od[t] == 0))), f"row {j}: distances differ"
        # rule 4: index sets equal up to ties at the k-th distance
        gs, os_ = set(g.tolist()), set(oi[t].tolist())
        if gs != os_ and kk > 0:
            dk = od[t][-1]
            diff = np.array(sorted(gs ^ os_), np.int64)
            dd = orc.distances(prims, kind, q[j], diff)
            bad = diff[~(np.abs(dd - dk) <= REL * max(dk, 1e-300))]
            assert bad.size == 0, f"row {j}: non-tie index mismatch {bad[:5]}"
            exempt += diff.size
        # rows come sorted by (distance, index): non-decreasing float distances
        assert np.all(np.diff(gpu_dist[j]) >= 0), f"row {j}: not ascending"
    return exempt


# ---------------------------------------------------------------- trees
def _karras_numbering(rows, refs, n, inv):
    """Node rows of a depth-first numbered tree (root 0, left child next,
    right child after the left subtree) moved to the Karras numbering (root
    0, the children of a node split at gamma are nodes gamma and gamma+1),
    with internal child references rewritten; leaf references (~primitive)
    are kept.  `inv` maps primitive -> sorted position."""
    ni = rows.shape[0]
    kid = np.full(ni, -1, np.int64)
    kid[0] = 0
    cur, lo = np.array([0], np.int64), np.array([0], np.int64)
    while cur.size:
        lr, rr = refs[cur, 0], refs[cur, 1]
        gamma = np.where(lr < 0, inv[np.clip(~lr, 0, n - 1)],
                         np.where(rr < 0, inv[np.clip(~rr, 0, n - 1)] - 1, rr - cur - 1 + lo))
        ml, mr = lr >= 0, rr >= 0
        kid[lr[ml]] = gamma[ml]
        kid[rr[mr]] = gamma[mr] + 1
        cur = np.concatenate([lr[ml], rr[mr]])
        lo = np.concatenate([lo[ml], gamma[mr] + 1])
    assert np.array_equal(np.sort(kid), np.arange(ni)), "depth-first numbering is not a tree order"
    new_refs = np.where(refs >= 0, kid[np.clip(refs, 0, ni - 1)], refs)
    out = np.empty_like(rows)
    out[kid] = rows
    out_refs = np.empty_like(new_refs)
    out_refs[kid] = new_refs
    return out, out_refs


def decode_tree(bvh):
    """Child kinds/indices (leaves by sorted position, as the hierarchy
    numbers them), permutation, node boxes and (for Q16) exact leaf boxes
    in sorted order, read back from device memory.  Leaf references name
    the primitive (~index); they are mapped back through the permutation."""
    lay = bvh.layout
    n = bvh.n
    ni = max(n - 1, 0)
    nodes = bvh.nodes_bytes().cpu().numpy()
    leaves = bvh.leaves_bytes().cpu().numpy()
    out = {}
    if lay.node_format == 0:
        f = nodes.view(np.float32).reshape(ni, 16)
        refs = nodes.view(np.int32).reshape(ni, 16)[:, 12:14]
        out["boxes_l"] = f[:, 0:6].copy()
        out["boxes_r"] = f[:, 6:12].copy()
        out["perm"] = leaves.view(np.int32).astype(np.int64)
    else:
        if bvh.kind == 0:
            out["perm"] = leaves.view(np.int32).astype(np.int64)
        else:
            rec = leaves.view(np.float32).reshape(n, 8)
            pos = leaves.view(np.int32).reshape(n, 8)[:, 6].astype(np.int64)
            perm = np.full(n, -1, np.int64)
            perm[pos] = np.arange(n)
            out["perm"] = perm
            out["leaf_boxes"] = rec[perm, :6].copy()
        if getattr(lay, "node_order", 0) == 2 and ni > 0:   # depth-first
            inv0 = np.full(n, 0, np.int64)
            inv0[out["perm"]] = np.arange(n)
            rows, r2 = _karras_numbering(nodes.reshape(ni, 32), nodes.view(np.int32).reshape(ni, 8)[:, 6:8]
                                         .astype(np.int64), n, inv0)
            rows = rows.copy()
            rows.view(np.int32).reshape(ni, 8)[:, 6:8] = r2.astype(np.int32)
            nodes = rows.reshape(-1)
        u = nodes.view(np.uint16).reshape(ni, 16)
        refs = nodes.view(np.int32).reshape(ni, 8)[:, 6:8]
        out["q_l"] = u[:, 0:6].astype(np.uint32)
        out["q_r"] = u[:, 6:12].astype(np.uint32)
    perm = out["perm"]
    inv = np.full(n, -1, np.int64)
    ok = (perm >= 0) & (perm < n)
    inv[perm[ok]] = np.nonzero(ok)[0]
    refs = refs.astype(np.int64)
    out["child_kind"] = (refs >= 0).astype(np.int8)
    out["child_index"] = np.where(refs >= 0, refs, inv[np.clip(~refs, 0, max(n - 1, 0))])
    if lay.node_format == 1 and bvh.kind == 0:
        # a point leaf's slot holds the float32 point
        f = nodes.view(np.float32).reshape(ni, 8)
        lb = np.full((n, 6), np.nan, np.float32)
        if n == 1:
            lb[0] = np.array(bvh.scene, np.float32)
        for s in range(2):
            m = refs[:, s] < 0
            xyz = f[m, 3 * s:3 * s + 3]
            lb[out["child_index"][m, s]] = np.concatenate([xyz, xyz], axis=1)
        out["leaf_boxes"] = lb
    return out


def fmaf32(q, scale, origin):
    """float32 fmaf(q, scale, origin), correctly rounded, vectorised.

    q * scale is exact in float64 (16-bit by 24-bit significands); adding
    origin in float64 rounds once more, which can only change the final
    float32 rounding when the float64 sum lands exactly on a float32
    midpoint -- those rare cases are redone with exact rationals."""
    from fractions import Fraction
    q = np.asarray(q, np.float64)
    s = np.float64(np.float32(scale))
    o = np.float64(np.float32(origin))
    v = q * s + o
    f = v.astype(np.float32)
    lo = np.nextafter(f, np.float32(-np.inf))
    hi = np.nextafter(f, np.float32(np.inf))
    mid = (v == (f.astype(np.float64) + lo.astype(np.float64)) / 2) | \
          (v == (f.astype(np.float64) + hi.astype(np.float64)) / 2)
    for i in zip(*np.nonzero(mid)):
        exact = Fraction(float(q[i])) * Fraction(float(s)) + Fraction(float(o))
        cands = [f[i], lo[i], hi[i]]
        err = [abs(Fraction(float(c)) - exact) for c in cands]
        best = min(err)
        pick = [c for c, e in zip(cands, err) if e == best]
        if len(pick) > 1:   # tie: even significand
            pick = [c for c in pick if (np.array(c, np.float32).view(np.uint32) & 1) == 0]
        f[i] = pick[0]
    return f


def dequantise(qbox, origin, scale):
    """Dequantised [.., 6] boxes, per the traversal's fmaf(q, scale, origin)."""
    out = np.empty(qbox.shape, np.float32)
    for c in range(6):
        a = c % 3
        out[..., c] = fmaf32(qbox[..., c], scale[a], origin[a])
    return out


# ---------------------------------------------------------------- 4-wide trees
EMPTY_REF = -2 ** 31


def expected_wide(ref, prims, kind, n):
    """The oracle's binary hierarchy collapsed at even depths: each internal
    node at even depth keeps its children's children (a leaf child stays a
    leaf child), numbered in depth-first order (left subtree first).
    Returns (refs int64 [W, 4]: node index, ~primitive for a leaf, EMPTY_REF
    for an unused slot; exact child boxes float32 [W, 4, 6], NaN when unused)."""
    ni = n - 1
    ck, ci, perm = ref["child_kind"], ref["child_index"], ref["perm"]
    sp = np.asarray(prims, np.float32).reshape(n, -1)[perm]
    leafbox = np.concatenate([sp[:, :3], sp[:, :3]], axis=1) if kind == 0 else sp
    depth = np.zeros(ni, np.int64)
    order = []
    stack = [0]
    while stack:
        u = stack.pop()
        order.append(u)
        for s in (1, 0):   # left child popped first
            if ck[u, s] == 1:
                depth[ci[u, s]] = depth[u] + 1
                stack.append(ci[u, s])
    even = [u for u in order if depth[u] % 2 == 0]
    widx = np.full(ni, -1, np.int64)
    widx[np.array(even, np.int64)] = np.arange(len(even))
    refs = np.full((len(even), 4), EMPTY_REF, np.int64)
    cbox = np.full((len(even), 4, 6), np.nan, np.float32)
    for w, u in enumerate(even):
        slots = []
        for s in (0, 1):
            if ck[u, s] == 0:
                slots.append((0, ci[u, s]))
            else:
                c = ci[u, s]
                slots.extend((int(ck[c, s2]), ci[c, s2]) for s2 in (0, 1))
        for j, (internal, x) in enumerate(slots):
            if internal:
                refs[w, j] = widx[x]
                cbox[w, j] = ref["boxes"][x]
            else:
                refs[w, j] = ~perm[x]
                cbox[w, j] = leafbox[x]
    return refs, cbox


def check_wide_tree(orc, prims, kind, bits, bvh):
    """A 4-wide tree against the oracle's hierarchy collapsed at even depths:
    the same node count, the same references slot by slot, point leaves'
    exact coordinates, every quantised slot containing its exact box, and the
    leaf region (permutation, or the exact box records of a box tree)."""
    n = bvh.n
    ref = orc.build(prims, kind, bits)
    lay = bvh.layout
    leaves = bvh.leaves_bytes().cpu().numpy()
    if kind == 0:
        assert np.array_equal(leaves.view(np.int32).astype(np.int64), ref["perm"])
    else:
        rec = leaves.view(np.float32).reshape(n, 8)
        np.testing.assert_array_equal(rec[:, :6], np.asarray(prims, np.float32).reshape(n, 6))
        pos = leaves.view(np.int32).reshape(n, 8)[:, 6].astype(np.int64)
        assert np.array_equal(ref["perm"][pos], np.arange(n))
    if n < 2:
        assert int(lay.node_count) == 0
        return
    want_refs, want_box = expected_wide(ref, prims, kind, n)
    W = want_refs.shape[0]
    assert int(lay.node_count) == W
    raw = bvh.nodes_bytes().cpu().numpy()
    assert raw.size == 64 * W
    refs = raw.view(np.int32).reshape(W, 16)[:, 12:16].astype(np.int64)
    assert np.array_equal(refs, want_refs)
    u16 = raw.view(np.uint16).reshape(W, 32)
    f32 = raw.view(np.float32).reshape(W, 16)
    for j in range(4):
        used = refs[:, j] != EMPTY_REF
        pleaf = used & (refs[:, j] < 0) & (kind == 0)
        np.testing.assert_array_equal(f32[pleaf, 3 * j:3 * j + 3], want_box[pleaf, j, :3])
        qs = used & ~pleaf
        d = dequantise(u16[qs, 6 * j:6 * j + 6].astype(np.uint32), list(lay.q16_origin),
                       list(lay.q16_scale))
        bad = ~(np.all(d[:, :3] <= want_box[qs, j, :3], axis=1) & np.all(d[:, 3:] >= want_box[qs, j, 3:], axis=1))
        assert not bad.any(), (f"slot {j}: quantised box not outward at nodes {np.nonzero(qs)[0][bad][:4]}: "
                               f"codes {u16[qs, 6 * j:6 * j + 6][bad][:2]}, dequantised {d[bad][:2]}, "
                               f"exact {want_box[qs, j][bad][:2]}, origin {list(lay.q16_origin)}, "
                               f"scale {list(lay.q16_scale)}")
