"""Parity at the full sizes of the benchmark workloads, through the same calls
the benchmark times (Morton-ordered queries, default visit budget, the
forest's tuned and graph-captured launch, the serving loop), on sampled rows
that the brute-force oracle answers one by one.

C3 rows are stratified: random queries plus those nearest the centre (the
heaviest nearest walks, which go to the cooperative pass), the corners
(farthest from the shell) and the shell itself (the only queries with radius
hits)."""
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


@pytest.mark.parametrize("fmt", ["fp32", "q16"])
def test_full_C2(orc, fmt):
    pts, q = datagen.config_inputs("C2")
    rows = np.sort(np.random.default_rng(21).choice(len(q), 400, replace=False))
    ex, total = run_config(orc, pts, q, datagen.CONFIGS["C2"]["radius"], fmt, rows)
    # about ten neighbours per query on average (radius from the density)
    assert 9.0e6 < total < 1.07e7
    assert ex <= 5


@pytest.fixture(scope="module")
def c3():
    pts, q = datagen.config_inputs("C3")
    nrm = np.linalg.norm(q.astype(np.float64), axis=1)
    rng = np.random.default_rng(31)
    near_shell = np.nonzero(np.abs(nrm - 1.0) < 2e-3)[0]
    rows = np.concatenate([rng.choice(len(q), 150, replace=False),
                           np.argpartition(nrm, 25)[:25],
                           np.argpartition(-nrm, 25)[:25],
                           rng.choice(near_shell, 60, replace=False)])
    return pts, q, np.unique(rows)


@pytest.mark.parametrize("fmt", ["fp32", "q16"])
def test_full_C3(orc, c3, fmt):
    pts, q, rows = c3
    ex, total = run_config(orc, pts, q, datagen.CONFIGS["C3"]["radius"], fmt, rows)
    assert 3.5e5 < total < 5.5e5    # ~4.3e5 hits, from the queries near the shell
    assert ex <= 2


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
    reqs = datagen.request_stream(24, 777, 1000.0, 4)
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
        rows = np.unique(np.linspace(0, m - 1, min(m, 12)).astype(np.int64))
        p = prims[r["tree"]]
        if r["kind"] == "radius":
            so, si = sub_csr(out["offsets"], out["indices"], rows)
            check_spatial(orc, p, 0, r["q"][rows], orc.WITHIN, so, si, radius=radii[r["tree"]])
        else:
            k = r["kind"]
            check_nearest(orc, p, 0, r["q"][rows], k, out["indices"].reshape(m, k)[rows],
                          out["distances"].reshape(m, k)[rows])
