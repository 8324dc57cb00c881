"""GPU parity on the paper's two experimental cases (section 3): filled
(filled-sphere queries in a filled-cube cloud) and hollow (hollow-sphere
queries in a hollow-cube cloud), radius r = (60/pi)^(1/3) and k = 10, with
the query ordering on and off.  Runs only on an MI355X (marker `gpu`)."""
import math

import numpy as np
import pytest
import torch

from paper_1908_11807_amd import abx, datagen
from parity import check_nearest, check_spatial

pytestmark = pytest.mark.gpu

P = 100_000
R = (60 / math.pi) ** (1 / 3)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("case", ["filled", "hollow"])
@pytest.mark.parametrize("fmt", ["fp32", "q16"])
def test_paper_case_parity_and_ordering(orc, case, fmt):
    if case == "filled":
        src, q = datagen.paper_filled_cube(P, 601), datagen.paper_filled_sphere(P, 602)
    else:
        src, q = datagen.paper_hollow_cube(P, 603), datagen.paper_hollow_sphere(P, 604)
    t = abx.bvh_build(dev(src), node_format=fmt)
    rows = np.random.default_rng(5).choice(P, 400, replace=False)
    res = {}
    for srt in (True, False):
        off, idx = abx.query_spatial(t, dev(q), radius=R, sort_queries=srt)
        _, ki, kd = abx.query_nearest(t, dev(q), 10, sort_queries=srt)
        res[srt] = (host(off), host(idx), host(ki), host(kd))
    off, idx, ki, kd = res[True]
    check_spatial(orc, src, 0, q, orc.WITHIN, off, idx, radius=R, rows=rows)
    check_nearest(orc, src, 0, q, 10, ki, kd, rows=rows)
    # the ordering changes the schedule, not the answer
    o2, i2, k2, d2 = res[False]
    assert np.array_equal(off, o2)
    for i in rows:
        assert set(idx[off[i]:off[i + 1]]) == set(i2[o2[i]:o2[i + 1]])
    assert np.array_equal(ki, k2) and np.array_equal(kd, d2)
    counts = np.diff(off)
    if case == "filled":
        # section 3: about 10 neighbours on average in the filled case
        assert abs(counts.mean() - 10.0) < 0.5
    else:
        # hollow: most queries find little, a few near the faces' centres many
        assert counts.mean() < 5.0 and counts.max() > 20 and np.median(counts) <= 2
