"""Parity at the full sizes of the benchmark workloads, through the same calls
the benchmark times (Morton-ordered queries, default visit budget, the
forest's tuned and graph-captured launch, the serving loop).

Two kinds of evidence, together covering every row:

* sampled rows that the brute-force oracle answers one by one (20 000 random
  C2 rows; 4 000 stratified C3 rows: random queries plus those nearest the
  centre -- the heaviest nearest walks, which go to the cooperative pass --,
  the corners, farthest from the shell, and the shell itself, the only
  queries with radius hits);
* on all rows, the equalities that the exactness argument of the method
  makes bitwise (section 2.2: the tree only prunes, so every variant returns
  the same rows): FP32 nodes = Q16 nodes, Morton-ordered = caller-ordered
  queries, two builds of the same input = the same tree bytes, the batched
  forest = 256 separate trees, a served request = the direct call; and
  properties that hold at any size: each nearest row is distinct, valid,
  sorted by distance, its distances agree with a float64
  recomputation, the radius search at the row's k-th distance returns a
  superset and slightly below it a subset of the row, and each radius pair
  lies within the radius in float64."""
import numpy as np
import pytest
import torch

from paper_1908_11807_amd import abx, datagen
from parity import check_nearest, check_spatial

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def sub_csr(off, idx, rows):
    """The CSR rows `rows` of (off, idx) (host arrays), as their own CSR."""
    off = np.asarray(off, np.int64)
    parts = [np.asarray(idx[off[r]:off[r + 1]]) for r in rows]
    so = np.concatenate([[0], np.cumsum([len(p) for p in parts])]).astype(np.int64)
    si = np.concatenate(parts) if parts else np.zeros(0, np.int32)
    return so, si


def run_config(orc, pts, q, radius, fmt, rows, k=10):
    t = abx.bvh_build(dev(pts), node_format=fmt)
    qd = dev(q)
    off, idx = abx.query_spatial(t, qd, radius=radius)
    _, ki, kd = abx.query_nearest(t, qd, k)
    torch.cuda.synchronize()
    off_h = off.cpu().numpy()
    assert off_h[0] == 0 and np.all(np.diff(off_h) >= 0) and off_h[-1] == idx.numel()
    so, si = sub_csr(off_h, idx.cpu().numpy(), rows)
    ex = check_spatial(orc, pts, 0, q[rows], orc.WITHIN, so, si, radius=radius)
    r = torch.from_numpy(rows).cuda()
    check_nearest(orc, pts, 0, q[rows], k, ki[r].cpu().numpy(), kd[r].cpu().numpy())
    return ex, int(off_h[-1])


# C2 names FP32 nodes: the large sample runs on them, a smaller one on Q16
@pytest.mark.parametrize("fmt,n_rows", [("fp32", 20_000), ("q16", 400)])
def test_full_C2(orc, fmt, n_rows):
    pts, q = datagen.config_inputs("C2")
    rows = np.sort(np.random.default_rng(21).choice(len(q), n_rows, replace=False))
    print(f"C2 {fmt}: {n_rows} oracle rows", flush=True)
    ex, total = run_config(orc, pts, q, datagen.CONFIGS["C2"]["radius"], fmt, rows)
    # about ten neighbours per query on average (radius from the density)
    assert 9.0e6 < total < 1.07e7
    assert ex <= 5 * max(1, n_rows // 400)


def c3_rows(q, seed, n_random, n_centre, n_corner, n_shell):
    nrm = np.linalg.norm(q.astype(np.float64), axis=1)
    rng = np.random.default_rng(seed)
    near_shell = np.nonzero(np.abs(nrm - 1.0) < 2e-3)[0]
    rows = np.concatenate([rng.choice(len(q), n_random, replace=False),
                           np.argpartition(nrm, n_centre)[:n_centre],
                           np.argpartition(-nrm, n_corner)[:n_corner],
                           rng.choice(near_shell, n_shell, replace=False)])
    return np.unique(rows)


@pytest.fixture(scope="module")
def c3():
    pts, q = datagen.config_inputs("C3")
    return pts, q


# the benchmark's Q16 nodes get the large stratified sample; FP32 nodes a
# smaller one (every row of the two is compared bitwise below)
@pytest.mark.parametrize("fmt,sample", [("q16", (2000, 500, 500, 1000)), ("fp32", (150, 25, 25, 60))])
def test_full_C3(orc, c3, fmt, sample):
    pts, q = c3
    rows = c3_rows(q, 31, *sample)
    print(f"C3 {fmt}: {len(rows)} oracle rows", flush=True)
    ex, total = run_config(orc, pts, q, datagen.CONFIGS["C3"]["radius"], fmt, rows)
    assert 3.5e5 < total < 5.5e5    # ~4.3e5 hits, from the queries near the shell
    assert ex <= 2 * max(1, len(rows) // 260)


# ------------------------------------------------------------ every row
def csr_keys(off, idx, n):
    """(row, index) pairs of a CSR on the device as int64 keys row * n + index."""
    off = off.to(torch.int64)
    rows = torch.repeat_interleave(torch.arange(off.numel() - 1, device=off.device), off[1:] - off[:-1])
    return rows * n + idx.to(torch.int64)


def in_keys(a, b):
    """Boolean mask: which keys of `a` occur in `b`."""
    if b.numel() == 0:
        return torch.zeros_like(a, dtype=torch.bool)
    bs = torch.sort(b).values
    pos = torch.searchsorted(bs, a).clamp_(max=bs.numel() - 1)
    return bs[pos] == a


def same_row_sets(off_a, idx_a, off_b, idx_b, n):
    if not torch.equal(off_a, off_b):
        return False
    ka = torch.sort(csr_keys(off_a, idx_a, n)).values
    kb = torch.sort(csr_keys(off_b, idx_b, n)).values
    return torch.equal(ka, kb)


def ulps(x, steps):
    """x moved by |steps| float32 ulps (up for steps > 0)."""
    toward = torch.full_like(x, float("inf") if steps > 0 else float("-inf"))
    for _ in range(abs(steps)):
        x = torch.nextafter(x, toward)
    return x


@pytest.fixture(scope="module")
def c3_runs(c3):
    """Radius and nearest results at C3 for both node formats (Morton-ordered
    queries, as timed) and for Q16 with the queries in the caller's order."""
    pts, q = c3
    r = datagen.CONFIGS["C3"]["radius"]
    qd = dev(q)
    out = {}
    for fmt in ("q16", "fp32"):
        print(f"C3 every row: {fmt}", flush=True)
        t = abx.bvh_build(dev(pts), node_format=fmt)
        off, idx = abx.query_spatial(t, qd, radius=r)
        _, ki, kd = abx.query_nearest(t, qd, 10)
        out[fmt] = dict(tree=t, off=off, idx=idx, ki=ki, kd=kd)
        if fmt == "q16":
            off_u, idx_u = abx.query_spatial(t, qd, radius=r, sort_queries=False)
            _, ki_u, kd_u = abx.query_nearest(t, qd, 10, sort_queries=False)
            out["q16_unsorted"] = dict(off=off_u, idx=idx_u, ki=ki_u, kd=kd_u)
        else:
            del t, out[fmt]["tree"]
    torch.cuda.synchronize()
    return out


def test_C3_every_row_fp32_equals_q16(c3, c3_runs):
    n = c3[0].shape[0]
    a, b = c3_runs["q16"], c3_runs["fp32"]
    assert torch.equal(a["ki"], b["ki"]) and torch.equal(a["kd"], b["kd"])
    assert same_row_sets(a["off"], a["idx"], b["off"], b["idx"], n)


def test_C3_every_row_sorted_equals_unsorted(c3, c3_runs):
    n = c3[0].shape[0]
    a, b = c3_runs["q16"], c3_runs["q16_unsorted"]
    assert torch.equal(a["ki"], b["ki"]) and torch.equal(a["kd"], b["kd"])
    assert same_row_sets(a["off"], a["idx"], b["off"], b["idx"], n)


def test_C3_build_is_deterministic(c3, c3_runs):
    pts = c3[0]
    a = c3_runs["q16"]["tree"]
    b = abx.bvh_build(dev(pts), node_format="q16")
    torch.cuda.synchronize()
    assert a.height == b.height and a.scene == b.scene
    assert torch.equal(a.nodes_bytes(), b.nodes_bytes())
    assert torch.equal(a.leaves_bytes(), b.leaves_bytes())


def test_C3_every_nearest_row_properties(c3, c3_runs):
    pts, q = c3
    n, m, k = pts.shape[0], q.shape[0], 10
    res = c3_runs["q16"]
    ki, kd = res["ki"], res["kd"]
    # distinct valid indices, distances non-decreasing (rows are ordered by
    # squared distance, then index; the reported square roots of two
    # different squares may round to one value, so index order is not
    # checked on equal reported distances)
    assert bool(((ki >= 0) & (ki < n)).all())
    srt = torch.sort(ki, dim=1).values
    assert bool((srt[:, 1:] != srt[:, :-1]).all())
    assert bool((kd[:, 1:] >= kd[:, :-1]).all())
    # reported float32 distances against a float64 recomputation
    p64 = dev(pts).double()
    q64 = dev(q).double()
    for s in range(0, m, 1_000_000):
        e = min(m, s + 1_000_000)
        d64 = torch.linalg.norm(p64[ki[s:e].long()] - q64[s:e, None, :], dim=2)
        g = kd[s:e].double()
        assert bool((torch.abs(g - d64) <= 1e-6 * torch.maximum(g, d64)).all()), s
    # the radius search at the k-th distance (a few ulps above) holds the
    # whole row; a few ulps below, only members of the row
    t = c3_runs["q16"]["tree"]
    qd = dev(q)
    hi = ulps(kd[:, -1].contiguous(), 4)
    lo = ulps(kd[:, -1].contiguous(), -4)
    off_hi, idx_hi = abx.query_spatial(t, qd, radii=hi)
    row_keys = (torch.arange(m, device=ki.device)[:, None] * n + ki.long()).reshape(-1)
    assert bool(in_keys(row_keys, csr_keys(off_hi, idx_hi, n)).all())
    assert bool(((off_hi[1:] - off_hi[:-1]) >= k).all())
    del off_hi, idx_hi
    off_lo, idx_lo = abx.query_spatial(t, qd, radii=lo)
    assert bool(in_keys(csr_keys(off_lo, idx_lo, n), row_keys).all())
    assert bool(((off_lo[1:] - off_lo[:-1]) < k).all())


def test_C3_every_radius_row_properties(c3, c3_runs):
    pts, q = c3
    n = pts.shape[0]
    r = datagen.CONFIGS["C3"]["radius"]
    res = c3_runs["q16"]
    off, idx = res["off"].long(), res["idx"].long()
    rows = torch.repeat_interleave(torch.arange(q.shape[0], device=off.device), off[1:] - off[:-1])
    p64, q64 = dev(pts).double(), dev(q).double()
    d64 = torch.linalg.norm(p64[idx] - q64[rows], dim=1)
    # every pair lies in the closed ball, up to the exemption band
    assert bool((d64 <= r * (1 + 1e-6)).all())
    # each nearest neighbour clearly inside the ball is in the radius row, and
    # each radius hit clearly nearer than the k-th neighbour is in the nearest row
    ki, kd = res["ki"].long(), res["kd"]
    kd64 = torch.linalg.norm(p64[ki] - q64[:, None, :], dim=2)
    inside = kd64 < r * (1 - 1e-6)
    nn_keys = (torch.arange(q.shape[0], device=ki.device)[:, None] * n + ki)
    rad_keys = rows * n + idx
    assert bool(in_keys(nn_keys[inside], rad_keys).all())
    kth = kd64[:, -1]
    nearer = d64 < kth[rows] * (1 - 1e-6)
    assert bool(in_keys(rad_keys[nearer], nn_keys.reshape(-1)).all())


def test_full_C4_forest(orc):
    k = 16
    pts, off, qs, qoff = datagen.forest_inputs(256)
    side = torch.cuda.Stream()      # graphs are captured on a stream of their own
    with torch.cuda.stream(side):
        plan = abx.ForestPlan(dev(pts), off, dev(qs), qoff, k, node_format="q16")
        plan.check()
        plan.autotune()
        plan.capture(build=True)
        plan.replay()
        torch.cuda.synchronize()
        offsets, idx, dist = plan.results()
    sizes = np.diff(off)
    kk = np.minimum(k, sizes)
    want = np.concatenate([[0], np.cumsum(np.repeat(kk, np.diff(qoff)))])
    assert np.array_equal(offsets.cpu().numpy().astype(np.int64), want)
    # three rows of every tree: first, middle, last query
    for t in range(len(sizes)):
        m_t = int(qoff[t + 1] - qoff[t])
        rows = np.unique(np.array([0, m_t // 2, m_t - 1], np.int64))
        s = want[qoff[t] + rows]
        pos = torch.from_numpy((s[:, None] + np.arange(kk[t])[None, :]).reshape(-1)).cuda()
        ti = idx[pos].cpu().numpy().reshape(len(rows), kk[t])
        td = dist[pos].cpu().numpy().reshape(len(rows), kk[t])
        check_nearest(orc, pts[off[t]:off[t + 1]], 0, qs[qoff[t]:qoff[t + 1]][rows], k, ti, td)


def test_C4_every_row_forest_equals_separate_trees():
    """The batched forest (one arena, composite keys, one persistent launch)
    against 256 separate builds and queries of the plain path: bitwise on
    all rows."""
    k = 16
    pts, off, qs, qoff = datagen.forest_inputs(256)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        plan = abx.ForestPlan(dev(pts), off, dev(qs), qoff, k, node_format="q16")
        plan.check()
        plan.query()
        torch.cuda.synchronize()
        offsets, idx, dist = plan.results()
    offsets = offsets.cpu().numpy().astype(np.int64)
    print("C4 every row: 256 separate trees", flush=True)
    for t in range(len(off) - 1):
        p_t = dev(pts[off[t]:off[t + 1]])
        q_t = dev(qs[qoff[t]:qoff[t + 1]])
        tree = abx.bvh_build(p_t, node_format="q16")
        _, ti, td = abx.query_nearest(tree, q_t, k)
        s, e = offsets[qoff[t]], offsets[qoff[t + 1]]
        assert torch.equal(idx[s:e].reshape(ti.shape), ti), t
        assert torch.equal(dist[s:e].reshape(td.shape), td), t


def test_full_C5_serving(orc):
    n = 10_000_000
    prims, trees, radii, pools = [], [], [], []
    for t in range(4):
        if t < 2:
            p = datagen.uniform_cube(n, 501 + t)
            radii.append(float(np.float32(datagen.radius_for_density(n))))
            pools.append(datagen.uniform_cube(1_000_000, 601 + t))
        else:
            p = datagen.shell(n, 501 + t)
            radii.append(float(np.float32(datagen.radius_for_shell(n, 1e-3))))
            pools.append(datagen.uniform_cube(1_000_000, 601 + t, -1.0, 1.0))
        prims.append(p)
        trees.append(abx.bvh_build(dev(p), node_format="q16"))
    torch.cuda.synchronize()
    srv = abx.Server(slots=4, budget_bytes=2 << 30, host_bytes=2 << 30)
    tids = [srv.add_tree(t) for t in trees]
    reqs = datagen.request_stream(48, 777, 1000.0, 4)
    rng = np.random.default_rng(778)
    tickets = []
    for r in reqs:
        o = int(rng.integers(0, 1_000_000 - r["m"] + 1))
        r["q"] = pools[r["tree"]][o:o + r["m"]]
        if r["kind"] == "radius":
            tickets.append(srv.submit(tids[r["tree"]], abx.REQ_RADIUS, r["q"], radius=radii[r["tree"]]))
        else:
            tickets.append(srv.submit(tids[r["tree"]], abx.REQ_NEAREST, r["q"], k=r["kind"]))
    res = [srv.wait(tk) for tk in tickets]
    srv.close()
    for r, out in zip(reqs, res):
        assert out["status"] == abx.OK
        m = r["m"]
        # every row: the served result equals the direct call on the same tree
        tree, qd = trees[r["tree"]], dev(r["q"])
        if r["kind"] == "radius":
            d_off, d_idx = abx.query_spatial(tree, qd, radius=radii[r["tree"]])
            assert np.array_equal(out["offsets"], d_off.cpu().numpy())
            assert same_row_sets(torch.from_numpy(out["offsets"]).cuda(),
                                 torch.from_numpy(out["indices"]).cuda(), d_off, d_idx, n)
        else:
            _, d_i, d_d = abx.query_nearest(tree, qd, r["kind"])
            assert np.array_equal(out["indices"], d_i.cpu().numpy().reshape(-1))
            assert np.array_equal(out["distances"], d_d.cpu().numpy().reshape(-1))
        rows = np.unique(np.linspace(0, m - 1, min(m, 12)).astype(np.int64))
        p = prims[r["tree"]]
        if r["kind"] == "radius":
            so, si = sub_csr(out["offsets"], out["indices"], rows)
            check_spatial(orc, p, 0, r["q"][rows], orc.WITHIN, so, si, radius=radii[r["tree"]])
        else:
            k = r["kind"]
            check_nearest(orc, p, 0, r["q"][rows], k, out["indices"].reshape(m, k)[rows],
                          out["distances"].reshape(m, k)[rows])
