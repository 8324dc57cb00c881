"""Failure paths of the bounded waits between workgroups, forced from the
host.  The sort's decoupled look-back (section 2.1 "Sort the bounding boxes",
section 2.2 "Query ordering") gives up at its first unanswered poll once
abx_set_sort_spin_limit(0) is set; every kernel still ends normally, and each
caller either reports ABX_ERR_DEVICE (sort, build, forest check) or falls back
to the caller's query order, which gives the same results bit for bit."""
import numpy as np
import pytest
import torch

from paper_1908_11807_amd import abx, datagen

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.fixture
def forced_giveup():
    prev = abx.set_sort_spin_limit(0)
    try:
        yield
    finally:
        abx.set_sort_spin_limit(prev)


@pytest.mark.parametrize("key_bits", [30, 63])
def test_sort_reports_giveup(forced_giveup, key_bits):
    rng = np.random.default_rng(key_bits)
    keys = rng.integers(0, 2 ** key_bits, size=50_000, dtype=np.uint64)
    k = dev(keys.astype(np.uint32).view(np.int32)) if key_bits <= 32 else dev(keys.view(np.int64))
    print(f"sort give-up, key_bits={key_bits}, n=50000", flush=True)
    with pytest.raises(abx.AbxError) as e:
        abx.radix_sort_pairs(k, key_bits)
    assert e.value.status == abx.ERR_DEVICE


def test_single_tile_sort_needs_no_wait(forced_giveup):
    # one tile (at most 5120 keys of 32 bits) never waits, so it cannot give up
    keys = np.random.default_rng(3).integers(0, 2 ** 30, size=4096).astype(np.uint32)
    ko, vo = abx.radix_sort_pairs(dev(keys.view(np.int32)), 30)
    assert np.array_equal(vo.cpu().numpy(), np.argsort(keys, kind="stable"))


@pytest.mark.parametrize("fmt", ["fp32", "q16"])
@pytest.mark.parametrize("hierarchy", ["karras", "agglomerative"])
@pytest.mark.parametrize("kind", [0, 1])
def test_build_fails_with_device_error(forced_giveup, fmt, hierarchy, kind):
    pts = datagen.uniform_cube(30_000, 7)
    prims = pts if kind == 0 else datagen.boxes_around(pts, 8, 0.01)
    print(f"build give-up, fmt={fmt}, hierarchy={hierarchy}, kind={kind}", flush=True)
    with pytest.raises(abx.AbxError) as e:
        abx.bvh_build(dev(prims), kind=kind, node_format=fmt, hierarchy=hierarchy)
    assert e.value.status == abx.ERR_DEVICE
    # the next build with the default limit succeeds (nothing left behind)
    abx.set_sort_spin_limit(-1)
    t = abx.bvh_build(dev(prims), kind=kind, node_format=fmt, hierarchy=hierarchy)
    assert t.n == prims.shape[0]


def test_depth_first_build_fails_with_device_error(forced_giveup):
    pts = datagen.uniform_cube(20_000, 8)
    with pytest.raises(abx.AbxError) as e:
        abx.bvh_build(dev(pts), node_format="q16", node_order="depth_first")
    assert e.value.status == abx.ERR_DEVICE


def _rows(off, idx):
    off = off.cpu().numpy()
    idx = idx.cpu().numpy()
    return [np.sort(idx[off[i]:off[i + 1]]) for i in range(len(off) - 1)]


@pytest.mark.parametrize("fmt", ["fp32", "q16"])
def test_query_order_falls_back_to_input_order(forced_giveup, fmt):
    # 5000 points: one tile of 63-bit keys (5376 keys), so the build itself never waits
    pts = datagen.uniform_cube(5000, 9)
    t = abx.bvh_build(dev(pts), node_format=fmt)
    q = dev(datagen.uniform_cube(20_000, 10))   # four tiles of 30-bit query codes (5120 keys)
    r = float(np.float32(datagen.radius_for_density(5000)))
    print(f"query order give-up, fmt={fmt}", flush=True)
    _, i_s, d_s = abx.query_nearest(t, q, 10, sort_queries=True)
    _, i_u, d_u = abx.query_nearest(t, q, 10, sort_queries=False)
    assert torch.equal(i_s, i_u) and torch.equal(d_s, d_u)
    o_s, x_s = abx.query_spatial(t, q, radius=r, sort_queries=True)
    o_u, x_u = abx.query_spatial(t, q, radius=r, sort_queries=False)
    assert torch.equal(o_s, o_u)
    assert all(np.array_equal(a, b) for a, b in zip(_rows(o_s, x_s), _rows(o_u, x_u)))
    o_1, x_1, info = abx.query_spatial_1p(t, q, 16, radius=r, sort_queries=True)
    assert torch.equal(o_1, o_u)
    assert all(np.array_equal(a, b) for a, b in zip(_rows(o_1, x_1), _rows(o_u, x_u)))


def test_forest_check_reports_device_error(forced_giveup):
    sizes = [5000, 3000, 8000, 1]
    pts = np.concatenate([datagen.uniform_cube(n, 20 + i) for i, n in enumerate(sizes)])
    qs = np.concatenate([datagen.uniform_cube(100, 40 + i) for i in range(len(sizes))])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    qoff = np.arange(0, 100 * len(sizes) + 1, 100, dtype=np.int64)
    print("forest give-up", flush=True)
    plan = abx.ForestPlan(dev(pts), off, dev(qs), qoff, 8, "q16")
    with pytest.raises(abx.AbxError) as e:
        plan.check()
    assert e.value.status == abx.ERR_DEVICE
    plan.query()                 # walks nothing: the kernels read the failed status
    torch.cuda.synchronize()
    abx.set_sort_spin_limit(-1)
    plan.build()
    plan.check()
    plan.query()
    offsets, idx, dist = plan.results()
    torch.cuda.synchronize()
    assert int(offsets[-1]) == 8 * 100 * 3 + 1 * 100


def test_injected_launch_failure_is_reported_and_recovered():
    pts = datagen.uniform_cube(20_000, 50)
    q = dev(datagen.uniform_cube(5000, 51))
    t = abx.bvh_build(dev(pts), node_format="q16")
    want = abx.query_nearest(t, q, 8)
    abx.inject_fault(abx.FAULT_LAUNCH, 0)
    try:
        with pytest.raises(abx.AbxError) as e:
            abx.query_nearest(t, q, 8)
        assert e.value.status == abx.ERR_HIP
    finally:
        abx.inject_fault(abx.FAULT_LAUNCH, -1)
    got = abx.query_nearest(t, q, 8)
    assert all(torch.equal(a, b) for a, b in zip(want, got))


def test_injected_failure_in_one_served_request_leaves_the_others_intact():
    pts = datagen.shell(50_000, 52, 0.99, 1.01)
    t = abx.bvh_build(dev(pts), node_format="q16")
    qs = [datagen.uniform_cube(700, 60 + i, -1.0, 1.0) for i in range(6)]
    direct = [abx.query_nearest(t, dev(q), 8) for q in qs]
    torch.cuda.synchronize()
    s = abx.Server(slots=1, budget_bytes=64 << 20, host_bytes=64 << 20, merge_queries=-1)
    tid = s.add_tree(t)
    # the failing launch is the first kernel of one request's sequence; with
    # one slot and no merging the requests run one after another
    first = s.submit(tid, abx.REQ_NEAREST, qs[0], k=8)
    assert s.wait(first)["status"] == abx.OK
    abx.inject_fault(abx.FAULT_LAUNCH, 0)
    try:
        tickets = [s.submit(tid, abx.REQ_NEAREST, q, k=8) for q in qs[1:]]
        res = [s.wait(tk) for tk in tickets]
    finally:
        abx.inject_fault(abx.FAULT_LAUNCH, -1)
    st = s.stats()
    s.close()
    status = [r["status"] for r in res]
    assert status.count(abx.ERR_HIP) == 1 and status.count(abx.OK) == 4
    assert st["failed"] == 1
    for (_, di, dd), r in zip(direct[1:], res):
        if r["status"] == abx.OK:
            assert np.array_equal(r["indices"], di.cpu().numpy().reshape(-1))
            assert np.array_equal(r["distances"], dd.cpu().numpy().reshape(-1))
