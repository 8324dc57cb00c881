"""GPU parity of the one-pass (1P) spatial query against the CPU oracle and
against the two-pass path: one traversal when every query fits its buffer,
the two-pass fill after an overflow, the capacity hand-off, the edge cases.
Runs only on an MI355X (marker `gpu`)."""
import numpy as np
import pytest
import torch

from paper_1908_11807_amd import abx, datagen
from parity import check_spatial

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rows_equal(off_a, idx_a, off_b, idx_b):
    """Same offsets, and each row the same set (order within a row is free)."""
    assert np.array_equal(off_a, off_b)
    for i in range(off_a.shape[0] - 1):
        a = np.sort(idx_a[off_a[i]:off_a[i + 1]])
        b = np.sort(idx_b[off_b[i]:off_b[i + 1]])
        assert np.array_equal(a, b), f"row {i}"


@pytest.mark.parametrize("fmt", ["fp32", "q16"])
@pytest.mark.parametrize("sort", [True, False])
def test_onepass_matches_oracle_and_two_pass(orc, fmt, sort):
    pts, q = datagen.config_inputs("C1")
    r = datagen.CONFIGS["C1"]["radius"]
    t = abx.bvh_build(dev(pts), node_format=fmt)
    o2, i2 = abx.query_spatial(t, dev(q), radius=r, sort_queries=sort)
    o2, i2 = host(o2), host(i2)
    maxc = int(np.diff(o2).max())
    for bs, want_passes in ((maxc, 1), (maxc + 7, 1), (max(maxc - 3, 1), 2), (1, 2)):
        o1, i1, passes = abx.query_spatial_1p(t, dev(q), bs, radius=r, sort_queries=sort)
        o1, i1 = host(o1), host(i1)
        assert passes == want_passes, (bs, maxc, passes)
        rows_equal(o1, i1, o2, i2)
    check_spatial(orc, pts, 0, q, orc.WITHIN, o1, i1, radius=r)


def test_onepass_box_predicates_on_box_tree(orc):
    pts = datagen.clusters(30_011, 21)
    boxes = datagen.boxes_around(pts, 22, 0.004)
    qb = datagen.boxes_around(datagen.uniform_cube(5_003, 23), 24, 0.01)
    for fmt in ("fp32", "q16"):
        t = abx.bvh_build(dev(boxes), kind=1, node_format=fmt)
        o1, i1, passes = abx.query_spatial_1p(t, dev(qb), 16, predicate="intersects")
        check_spatial(orc, boxes, 1, qb, orc.INTERSECTS, host(o1), host(i1))
        o2, i2 = abx.query_spatial(t, dev(qb), predicate="intersects")
        rows_equal(host(o1), host(i1), host(o2), host(i2))


def test_onepass_per_query_radii_and_ragged_tail(orc):
    pts = datagen.uniform_cube(20_000, 31)
    q = datagen.uniform_cube(4_097, 32)          # ragged: 16 full tiles + 1
    radii = np.random.default_rng(33).uniform(0.0, 0.05, 4_097).astype(np.float32)
    radii[::97] = -1.0                           # negative radius: no hits
    t = abx.bvh_build(dev(pts), node_format="q16")
    o1, i1, _ = abx.query_spatial_1p(t, dev(q), 8, radii=dev(radii))
    check_spatial(orc, pts, 0, q, orc.WITHIN, host(o1), host(i1), radii=radii)
    assert np.all(np.diff(host(o1))[::97] == 0)


def test_onepass_capacity_hand_off(orc):
    pts, q = datagen.config_inputs("C1")
    r = datagen.CONFIGS["C1"]["radius"]
    t = abx.bvh_build(dev(pts))
    # an index buffer too small for the total: the call reports the total,
    # and the binding finishes with the fill entry point on the same scratch
    o1, i1, passes = abx.query_spatial_1p(t, dev(q), 64, radius=r, capacity=100)
    assert passes == 2
    o2, i2 = abx.query_spatial(t, dev(q), radius=r)
    rows_equal(host(o1), host(i1), host(o2), host(i2))


def test_onepass_empty_cases():
    t = abx.bvh_build(dev(datagen.uniform_cube(100, 41)))
    o, i, passes = abx.query_spatial_1p(t, dev(np.zeros((0, 3), np.float32)), 4, radius=0.1)
    assert host(o).tolist() == [0] and i.numel() == 0 and passes == 0
    far = np.full((10, 3), 50.0, np.float32)
    o, i, passes = abx.query_spatial_1p(t, dev(far), 4, radius=0.1)
    assert host(o).tolist() == [0] * 11 and passes == 1
    one = abx.bvh_build(dev(np.array([[0.5, 0.5, 0.5]], np.float32)), node_format="q16")
    o, i, _ = abx.query_spatial_1p(one, dev(np.array([[0.5, 0.5, 0.6], [0.9, 0.9, 0.9]], np.float32)),
                                   1, radius=0.2)
    assert host(o).tolist() == [0, 1, 1] and host(i).tolist() == [0]
