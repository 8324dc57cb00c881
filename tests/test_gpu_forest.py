"""GPU parity of the batched forest (many trees in one arena, one persistent
query launch, HIP-graph replay, autotuner) against the per-tree oracle."""
import numpy as np
import pytest
import torch

from paper_1908_11807_amd import abx, datagen
from parity import check_nearest

pytestmark = pytest.mark.gpu


def make_forest(seed, sizes, qsizes):
    pts, qs = [], []
    for t, (n, m) in enumerate(zip(sizes, qsizes)):
        gen = datagen.uniform_cube if t % 2 == 0 else datagen.clusters
        pts.append(gen(n, seed + t) if n else np.zeros((0, 3), np.float32))
        qs.append(gen(m, seed + 1000 + t) if m else np.zeros((0, 3), np.float32))
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    qoff = np.concatenate([[0], np.cumsum(qsizes)]).astype(np.int64)
    return np.concatenate(pts), off, np.concatenate(qs), qoff


def check_forest(orc, pts, off, qs, qoff, k, offsets, idx, dist, rows_per_tree=None):
    offsets = offsets.cpu().numpy().astype(np.int64)
    idx = idx.cpu().numpy()
    dist = dist.cpu().numpy()
    T = len(off) - 1
    total = 0
    for t in range(T):
        n_t = off[t + 1] - off[t]
        kk = min(k, n_t)
        for i in range(qoff[t], qoff[t + 1]):
            assert offsets[i] == total, (t, i)
            total += kk
        m_t = qoff[t + 1] - qoff[t]
        if m_t == 0 or kk == 0:
            continue
        rows = np.arange(m_t) if rows_per_tree is None else \
            np.unique(np.linspace(0, m_t - 1, min(m_t, rows_per_tree)).astype(np.int64))
        s = offsets[qoff[t]]
        ti = idx[s: s + m_t * kk].reshape(m_t, kk)
        td = dist[s: s + m_t * kk].reshape(m_t, kk)
        check_nearest(orc, pts[off[t]:off[t + 1]], 0, qs[qoff[t]:qoff[t + 1]], k, ti, td, rows=rows)
    assert offsets[-1] == total


@pytest.mark.parametrize("fmt", ["fp32", "q16"])
@pytest.mark.parametrize("k", [1, 10, 16, 40, 64])
def test_forest_nearest_matches_oracle(orc, fmt, k):
    sizes = [0, 1, 3, 9, 17, 100, 1000, 2500, 40, 5000, 1, 777]
    qsizes = [5, 7, 0, 30, 64, 65, 300, 129, 11, 400, 3, 250]
    pts, off, qs, qoff = make_forest(11, sizes, qsizes)
    plan = abx.ForestPlan(torch.from_numpy(pts).cuda(), off, torch.from_numpy(qs).cuda(), qoff, k, fmt)
    plan.check()
    plan.query()
    torch.cuda.synchronize()
    check_forest(orc, pts, off, qs, qoff, k, *plan.results())


def test_forest_cooperative_pass(orc):
    sizes = [20_000, 15_000, 3]
    qsizes = [500, 400, 9]
    pts = np.concatenate([datagen.shell(20_000, 1, 1 - 5e-3, 1 + 5e-3), datagen.clusters(15_000, 2),
                          datagen.uniform_cube(3, 3)])
    qs = np.concatenate([datagen.uniform_cube(500, 4, -1.0, 1.0), datagen.uniform_cube(400, 5),
                         datagen.uniform_cube(9, 6)])
    off = np.array([0, 20_000, 35_000, 35_003], np.int64)
    qoff = np.array([0, 500, 900, 909], np.int64)
    plan = abx.ForestPlan(torch.from_numpy(pts).cuda(), off, torch.from_numpy(qs).cuda(), qoff, 10, "q16")
    for budget in (1, 50, 1 << 40):
        plan.query(dict(blocks_per_cu=2, tiles_per_grab=2, budget=budget))
        torch.cuda.synchronize()
        check_forest(orc, pts, off, qs, qoff, 10, *plan.results())


def test_forest_graph_replays_match_eager():
    sizes = list(np.random.default_rng(3).integers(1, 3000, size=40))
    qsizes = list(np.random.default_rng(4).integers(0, 200, size=40))
    pts, off, qs, qoff = make_forest(21, sizes, qsizes)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        plan = abx.ForestPlan(torch.from_numpy(pts).cuda(), off, torch.from_numpy(qs).cuda(), qoff, 16)
        plan.query()
        torch.cuda.synchronize()
        ref = [x.clone() for x in plan.results()]
        plan.capture(build=True)
        for rep in range(3):
            for x in (plan.offsets, plan.indices, plan.distances):
                x.fill_(-7)                                  # eager work between replays
            torch.cuda.synchronize()
            plan.replay()
            torch.cuda.synchronize()
            got = plan.results()
            for a, b in zip(ref, got):
                assert torch.equal(a, b), f"replay {rep} differs"
    plan.check()


def test_forest_autotune_keeps_results(tmp_path):
    sizes = [3000] * 8
    qsizes = [500] * 8
    pts, off, qs, qoff = make_forest(31, sizes, qsizes)
    plan = abx.ForestPlan(torch.from_numpy(pts).cuda(), off, torch.from_numpy(qs).cuda(), qoff, 16)
    plan.query()
    torch.cuda.synchronize()
    ref = [x.clone() for x in plan.results()]
    path = tmp_path / "tune.json"
    cfg = plan.autotune(str(path))
    assert cfg["blocks_per_cu"] >= 1 and cfg["tiles_per_grab"] >= 1
    import json
    rec = json.loads(path.read_text().strip().splitlines()[-1])
    assert len(rec["candidates"]) >= 6 and rec["best"]["budget"] == cfg["budget"]
    plan.query()
    torch.cuda.synchronize()
    for a, b in zip(ref, plan.results()):
        assert torch.equal(a, b)


def test_forest_check_flags_nan():
    pts = datagen.uniform_cube(100, 1)
    pts[37, 2] = np.nan
    plan = abx.ForestPlan(torch.from_numpy(pts).cuda(), [0, 50, 100],
                          torch.from_numpy(datagen.uniform_cube(4, 2)).cuda(), [0, 2, 4], 3)
    with pytest.raises(abx.AbxError) as e:
        plan.check()
    assert e.value.status == abx.ERR_INVALID_INPUT


def test_forest_k_above_64_unsupported():
    pts, off, qs, qoff = make_forest(21, [100, 200], [10, 20])
    plan = abx.ForestPlan(torch.from_numpy(pts).cuda(), off, torch.from_numpy(qs).cuda(), qoff, 65, "q16")
    with pytest.raises(abx.AbxError) as e:
        plan.query()
    assert e.value.status == abx.ERR_UNSUPPORTED


def test_forest_stats_count_the_walks():
    # the counting walk: every query with a tree of two or more points visits
    # at least the root; point trees read no leaf records; an empty tree's
    # queries count nothing
    sizes = [0, 1, 2, 50, 3000, 777]
    qsizes = [4, 5, 6, 100, 200, 50]
    pts, off, qs, qoff = make_forest(31, sizes, qsizes)
    plan = abx.ForestPlan(torch.from_numpy(pts).cuda(), off, torch.from_numpy(qs).cuda(), qoff, 10, "q16")
    plan.check()
    st = plan.stats().cpu().numpy()
    assert st.shape == (int(qoff[-1]), 2)
    assert np.all(st[:, 1] == 0)
    tree = np.repeat(np.arange(len(sizes)), qsizes)
    n_t = np.array(sizes)[tree]
    assert np.all(st[n_t <= 1, 0] == 0)
    assert np.all(st[n_t >= 2, 0] >= 1)
    assert np.all(st[n_t >= 2, 0] <= np.maximum(n_t[n_t >= 2] - 1, 1))
