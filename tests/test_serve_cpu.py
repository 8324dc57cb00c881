"""The serving scheduler's admission, memory accounting and latency
bookkeeping, run without a GPU (simulated executor: each phase lasts
sim_ns_per_query * m ns; radius requests find 10 results per query)."""
import numpy as np
import pytest

from paper_1908_11807_amd import abx


def _server(**kw):
    # one request per launch unless a test asks for merging
    kw.setdefault("merge_queries", -1)
    s = abx.Server(simulate=True, **kw)
    s.add_tree(None)
    return s


def test_fifo_admission_and_slot_limit():
    s = _server(slots=3, budget_bytes=1 << 30, host_bytes=1 << 28, sim_ns_per_query=2000)
    q = np.zeros((500, 3), np.float32)
    tickets = [s.submit(0, abx.REQ_NEAREST, q, k=8) for _ in range(12)]
    res = [s.wait(t) for t in tickets]
    assert all(r["status"] == abx.OK for r in res)
    admits = [r["t_admit"] for r in res]
    assert admits == sorted(admits)                       # FIFO admission
    st = s.stats()
    assert st["max_in_flight"] <= 3 and st["completed"] == 12
    for r in res:
        assert r["t_arrival"] <= r["t_admit"] <= r["t_done"]
        assert r["t_done"] - r["t_admit"] >= 500 * 2000e-9 * 0.99
        # one phase of the simulated executor's length
        assert r["t_device"] == pytest.approx(500 * 2000e-9)
        assert r["offsets"].tolist() == list(range(0, 8 * 501, 8))
    for t in tickets:
        s.release(t)
    s.close()


def test_budget_pressure_limits_concurrency():
    # each nearest request of m=1000, k=8 reserves ~ 12m + scratch + 64m bytes;
    # a budget for about two of them keeps at most two in flight
    s = _server(slots=8, budget_bytes=300_000, host_bytes=1 << 26, sim_ns_per_query=1000)
    q = np.zeros((1000, 3), np.float32)
    tickets = [s.submit(0, abx.REQ_NEAREST, q, k=8) for _ in range(10)]
    res = [s.wait(t) for t in tickets]
    st = s.stats()
    assert all(r["status"] == abx.OK for r in res)
    assert 1 <= st["max_in_flight"] <= 2
    assert st["device_high_water"] <= 300_000
    s.close()


def test_request_larger_than_budget_fails_alone():
    s = _server(slots=2, budget_bytes=100_000, host_bytes=1 << 26, sim_ns_per_query=100)
    small = np.zeros((10, 3), np.float32)
    big = np.zeros((100_000, 3), np.float32)
    t1 = s.submit(0, abx.REQ_NEAREST, small, k=4)
    t2 = s.submit(0, abx.REQ_NEAREST, big, k=4)
    t3 = s.submit(0, abx.REQ_NEAREST, small, k=4)
    assert s.wait(t1)["status"] == abx.OK
    assert s.wait(t2)["status"] == abx.ERR_CAPACITY
    assert s.wait(t3)["status"] == abx.OK                  # the queue moves on
    s.close()


def test_radius_two_phases_and_host_release_backpressure():
    # host arena holds only a few results: later requests wait until the
    # caller releases earlier ones.  With four slots requests can complete
    # out of submission order, and a fill may wait for space held by a
    # later request's results, so the caller releases in completion order
    # (waiting in submission order could wait on itself)
    s = _server(slots=4, budget_bytes=1 << 30, host_bytes=64 * 1024, sim_ns_per_query=100)
    q = np.zeros((200, 3), np.float32)
    tickets = [s.submit(0, abx.REQ_RADIUS, q, radius=0.1) for _ in range(20)]
    live, deadline = set(tickets), abx.server_now() + 60.0
    while live and abx.server_now() < deadline:
        for t in list(live):
            r = s.poll(t)
            if r is None:
                continue
            assert r["status"] == abx.OK and r["total"] == 10 * 200
            # count and fill phases; a count that was sent back to the queue
            # (its fill waited on the others' host space) ran once more
            phases = r["t_device"] / (200 * 100e-9)
            assert phases == pytest.approx(round(phases)) and round(phases) >= 2
            s.release(t)
            live.discard(t)
    assert not live, s.stats()
    assert s.stats()["host_high_water"] <= 64 * 1024
    s.close()


def test_latency_percentiles_accounting():
    s = _server(slots=2, budget_bytes=1 << 30, host_bytes=1 << 26, sim_ns_per_query=5000)
    now = abx.server_now()
    q = np.zeros((100, 3), np.float32)
    ts = [s.submit(0, abx.REQ_NEAREST, q, k=1, t_arrival=now) for _ in range(6)]
    lat = sorted(s.wait(t)["t_done"] - now for t in ts)
    # two slots, 0.5 ms per request: the i-th pair finishes after ~(i+1) * 0.5 ms
    assert lat[-1] >= 3 * 100 * 5000e-9 * 0.99
    s.close()


def test_submit_validation():
    s = _server(slots=1, budget_bytes=1 << 20, host_bytes=1 << 20)
    with pytest.raises(abx.AbxError):
        s.submit(5, abx.REQ_NEAREST, np.zeros((3, 3), np.float32), k=2)   # unknown tree
    with pytest.raises(abx.AbxError):
        s.submit(0, abx.REQ_NEAREST, np.zeros((3, 3), np.float32), k=129)  # k > 128
    s.close()


def test_fills_waiting_on_each_other_are_serialised():
    # A radius request of m = 1000 reserves ~58 KB for its count and then
    # 40 KB for its 10 000 simulated results.  Two counts fit the budget
    # together, but then neither fill fits beside the other's reservation:
    # the later request gives its reservation back and runs after the first.
    budget = 2 * 58_000 + 20_000
    s = _server(slots=4, budget_bytes=budget, host_bytes=1 << 26, sim_ns_per_query=100)
    q = np.zeros((1000, 3), np.float32)
    tickets = [s.submit(0, abx.REQ_RADIUS, q, radius=0.1) for _ in range(3)]
    deadline = abx.server_now() + 10.0
    res = {}
    while len(res) < len(tickets) and abx.server_now() < deadline:
        for t in tickets:
            if t not in res:
                r = s.poll(t)
                if r is not None:
                    res[t] = r
    assert len(res) == len(tickets), s.stats()          # no request is stuck
    for t in tickets:
        assert res[t]["status"] == abx.OK and res[t]["total"] == 10 * 1000
    st = s.stats()
    assert st["requeued"] >= 1 and st["device_high_water"] <= budget
    s.close()


def _batches(res):
    """Requests grouped by launch: the members of one batch share their
    admission time."""
    groups = {}
    for i, r in enumerate(res):
        groups.setdefault(r["t_admit"], []).append(i)
    return list(groups.values())


def test_small_requests_of_one_class_are_merged():
    # one slot busy with a long request; the small ones queued behind it
    # leave together as merged batches
    s = _server(slots=1, budget_bytes=1 << 30, host_bytes=1 << 28, sim_ns_per_query=2000,
                merge_queries=2000)
    q = np.zeros((500, 3), np.float32)
    first = s.submit(0, abx.REQ_NEAREST, np.zeros((5000, 3), np.float32), k=8)
    tickets = [s.submit(0, abx.REQ_NEAREST, q, k=8) for _ in range(12)]
    res = [s.wait(t) for t in tickets]
    assert s.wait(first)["status"] == abx.OK
    assert all(r["status"] == abx.OK for r in res)
    for r in res:
        assert r["offsets"].tolist() == list(range(0, 8 * 501, 8))
        # the batch's phase lasts for all its queries
        assert r["t_device"] >= 500 * 2000e-9 * 0.99
    groups = _batches(res)
    assert all(len(g) <= 4 for g in groups)               # 4 x 500 = the 2000-query limit
    assert len(groups) <= 4 and s.stats()["batches"] <= 5
    # batches keep the queue's order
    assert [g[0] for g in groups] == sorted(g[0] for g in groups)
    s.close()


def test_merging_keeps_classes_apart():
    s = _server(slots=1, budget_bytes=1 << 30, host_bytes=1 << 28, sim_ns_per_query=1000,
                merge_queries=1 << 20)
    s.add_tree(None)
    q = np.zeros((100, 3), np.float32)
    blocker = s.submit(0, abx.REQ_NEAREST, np.zeros((20_000, 3), np.float32), k=1)
    kinds = [(0, abx.REQ_NEAREST, 8, 0.0), (0, abx.REQ_NEAREST, 1, 0.0), (0, abx.REQ_RADIUS, 0, 0.1),
             (1, abx.REQ_NEAREST, 8, 0.0), (0, abx.REQ_RADIUS, 0, 0.2)]
    subs = [kinds[i % len(kinds)] for i in range(25)]
    tickets = [s.submit(tr, kd, q, k=k, radius=r) for tr, kd, k, r in subs]
    res = [s.wait(t) for t in tickets]
    s.wait(blocker)
    assert all(r["status"] == abx.OK for r in res)
    for g in _batches(res):
        assert len({subs[i] for i in g}) == 1                 # one class per launch
    assert len(_batches(res)) == len(kinds)                   # each class merged once
    for i, r in enumerate(res):
        if subs[i][1] == abx.REQ_RADIUS:
            assert r["total"] == 10 * 100
    s.close()


def test_small_requests_pass_a_blocked_large_one():
    # two slots: at most one large batch runs, so a second large request
    # waits and the small one behind it starts first
    s = _server(slots=2, budget_bytes=1 << 30, host_bytes=1 << 28, sim_ns_per_query=200,
                merge_queries=0, small_queries=1000, merge_large=-1)
    big = np.zeros((20_000, 3), np.float32)
    small = np.zeros((10, 3), np.float32)
    t1 = s.submit(0, abx.REQ_NEAREST, big, k=4)
    t2 = s.submit(0, abx.REQ_NEAREST, big, k=4)
    t3 = s.submit(0, abx.REQ_NEAREST, small, k=4)
    r1, r2, r3 = s.wait(t1), s.wait(t2), s.wait(t3)
    assert r1["status"] == r2["status"] == r3["status"] == abx.OK
    assert r3["t_admit"] < r2["t_admit"]                 # passed the waiting large one
    assert r3["t_done"] < r1["t_done"]
    assert r2["t_admit"] >= r1["t_done"] - 1e-3          # one large batch at a time
    s.close()


def test_large_requests_merge_when_queued_together():
    # large requests of one class that wait together run as one batch (up
    # to merge_large queries); a large request of another class does not
    # join, nor does one that would pass the limit
    s = _server(slots=1, budget_bytes=1 << 30, host_bytes=1 << 28, sim_ns_per_query=50,
                merge_queries=0, small_queries=1000, merge_large=50_000)
    big = np.zeros((20_000, 3), np.float32)
    t = [s.submit(0, abx.REQ_NEAREST, big, k=4) for _ in range(3)]
    other = s.submit(0, abx.REQ_NEAREST, big, k=5)
    rs = [s.wait(x) for x in t] + [s.wait(other)]
    assert all(r["status"] == abx.OK for r in rs)
    st = s.stats()
    # the first request runs alone (the scheduler admits it at once) or with
    # the second; the k = 5 request always alone: at most 3 batches of k = 4
    assert st["completed"] == 4 and st["batches"] <= 3
    # two requests of 20 000 share a batch: one admission for both
    admits = sorted(rs[i]["t_admit"] for i in range(3))
    assert admits[0] == admits[1] or admits[1] == admits[2]
    s.close()


def test_merged_radius_batches_with_host_backpressure():
    # merged radius batches still reserve each request's result space; the
    # caller releases results as they complete (with merging, a request can
    # complete before one submitted earlier, so an arena too small for the
    # results in flight needs releases in completion order)
    s = _server(slots=2, budget_bytes=1 << 30, host_bytes=96 * 1024, sim_ns_per_query=100,
                merge_queries=1000)
    q = np.zeros((200, 3), np.float32)
    tickets = [s.submit(0, abx.REQ_RADIUS, q, radius=0.1) for _ in range(20)]
    live, deadline = set(tickets), abx.server_now() + 20.0
    while live and abx.server_now() < deadline:
        for t in list(live):
            r = s.poll(t)
            if r is not None:
                assert r["status"] == abx.OK and r["total"] == 10 * 200
                s.release(t)
                live.discard(t)
    assert not live, s.stats()
    st = s.stats()
    assert st["host_high_water"] <= 96 * 1024 and st["completed"] == 20
    assert st["batches"] < 20
    s.close()


def test_injected_launch_failure_fails_one_request_only():
    # the third batch's launch fails: that request reports ABX_ERR_HIP, the
    # others complete with their results, and the server keeps serving
    s = _server(slots=1, budget_bytes=1 << 30, host_bytes=1 << 26, sim_ns_per_query=100)
    q = np.zeros((300, 3), np.float32)
    abx.inject_fault(abx.FAULT_LAUNCH, 2)
    try:
        tickets = [s.submit(0, abx.REQ_NEAREST, q, k=4) for _ in range(6)]
        res = [s.wait(t) for t in tickets]
    finally:
        abx.inject_fault(abx.FAULT_LAUNCH, -1)
    status = [r["status"] for r in res]
    assert status == [abx.OK, abx.OK, abx.ERR_HIP, abx.OK, abx.OK, abx.OK]
    for r in res:
        if r["status"] == abx.OK:
            assert r["offsets"].tolist() == list(range(0, 4 * 301, 4))
    st = s.stats()
    assert st["failed"] == 1 and st["completed"] == 5
    again = s.wait(s.submit(0, abx.REQ_RADIUS, q, radius=0.1))
    assert again["status"] == abx.OK and again["total"] == 3000
    s.close()


def test_injected_failure_fails_every_member_of_a_merged_batch():
    s = _server(slots=1, budget_bytes=1 << 30, host_bytes=1 << 26, sim_ns_per_query=2000,
                merge_queries=1 << 16)
    q = np.zeros((100, 3), np.float32)
    first = s.submit(0, abx.REQ_NEAREST, np.zeros((5000, 3), np.float32), k=2)
    deadline = abx.server_now() + 10.0
    while s.stats()["in_flight"] == 0 and abx.server_now() < deadline:
        pass                                    # until the first one has launched
    abx.inject_fault(abx.FAULT_LAUNCH, 0)       # the next launch: the merged batch
    try:
        tickets = [s.submit(0, abx.REQ_NEAREST, q, k=2) for _ in range(5)]
        res = [s.wait(t) for t in tickets]
    finally:
        abx.inject_fault(abx.FAULT_LAUNCH, -1)
    assert s.wait(first)["status"] == abx.OK
    assert all(r["status"] == abx.ERR_HIP for r in res)   # they ran as one batch
    assert s.stats()["failed"] == 5
    assert s.wait(s.submit(0, abx.REQ_NEAREST, q, k=2))["status"] == abx.OK
    s.close()


def test_injected_host_allocation_failure():
    abx.inject_fault(abx.FAULT_HOST_ALLOC, 0)
    try:
        with pytest.raises(abx.AbxError) as e:
            abx.Server(simulate=True, slots=1, budget_bytes=1 << 20, host_bytes=1 << 20)
        assert e.value.status == abx.ERR_HIP
    finally:
        abx.inject_fault(abx.FAULT_HOST_ALLOC, -1)
    s = _server(slots=1, budget_bytes=1 << 20, host_bytes=1 << 20)   # the next one works
    s.close()
    with pytest.raises(abx.AbxError):
        abx.inject_fault(7, 0)
