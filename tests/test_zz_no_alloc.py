"""abx_query_nearest_static, the nearest query that allocates nothing (its
scratch is the library's per-GPU array), against abx_query_nearest on the
same tree and queries: identical offsets, indices and distances, bit for bit,
on two calls in a row -- the second with fewer queries, so anything the
first left in the shared array would show -- and a batch beyond the array's
size refused before anything is launched."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1908_11807_amd import abx, datagen

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def scratch_bytes(t, m, k):
    sb = C.c_size_t()
    assert abx.library().abx_query_nearest_sizes(t.handle, m, k, C.byref(sb)) == abx.OK
    return sb.value


@pytest.mark.parametrize("fmt", ["fp32", "q16"])
@pytest.mark.parametrize("k", [1, 10, 32, 100])
def test_static_nearest_equals_plain(fmt, k):
    # cube queries against a shell: the central ones exceed the visit budget
    # and go through the cooperative pass and its saved walks in the scratch
    pts = datagen.shell(200_000, 71)
    t = abx.bvh_build(dev(pts), node_format=fmt)
    for m, seed, sort in ((300_000, 72, True), (50_000, 73, True), (20_000, 74, False)):
        assert scratch_bytes(t, m, k) <= abx.STATIC_SCRATCH_BYTES
        q = dev(datagen.uniform_cube(m, seed, -1.0, 1.0))
        print(f"static nearest: fmt={fmt} k={k} m={m} sort={sort}", flush=True)
        want = abx.query_nearest(t, q, k, sort_queries=sort)
        got = abx.query_nearest_static(t, q, k, sort_queries=sort)
        torch.cuda.synchronize()
        for a, b in zip(want, got):
            assert torch.equal(a, b)


def test_static_nearest_refuses_large_batches():
    pts = datagen.uniform_cube(10_000, 75)
    t = abx.bvh_build(dev(pts), node_format="q16")
    m = 2_000_000
    assert scratch_bytes(t, m, 10) > abx.STATIC_SCRATCH_BYTES
    q = torch.zeros((m, 3), dtype=torch.float32, device="cuda")
    out = (torch.full((m + 1,), -7, dtype=torch.int32, device="cuda"),
           torch.full((m, 10), -7, dtype=torch.int32, device="cuda"),
           torch.full((m, 10), -7.0, dtype=torch.float32, device="cuda"))
    with pytest.raises(abx.AbxError) as e:
        abx.query_nearest_static(t, q, 10, out=out)
    assert e.value.status == abx.ERR_CAPACITY
    torch.cuda.synchronize()
    assert bool((out[0] == -7).all()) and bool((out[1] == -7).all())


def test_static_nearest_empty_and_degenerate():
    t0 = abx.bvh_build(torch.zeros((0, 3), dtype=torch.float32, device="cuda"), node_format="q16")
    off, idx, dist = abx.query_nearest_static(t0, dev(datagen.uniform_cube(100, 76)), 10)
    torch.cuda.synchronize()
    assert idx.shape == (100, 0) and bool((off == 0).all())
    t1 = abx.bvh_build(dev(datagen.uniform_cube(1, 77)), node_format="fp32")
    q = dev(datagen.uniform_cube(5000, 78))
    for a, b in zip(abx.query_nearest(t1, q, 4), abx.query_nearest_static(t1, q, 4)):
        assert torch.equal(a, b)
