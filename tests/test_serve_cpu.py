"""The serving scheduler's admission, memory accounting and latency
bookkeeping, run without a GPU (simulated executor: each phase lasts
sim_ns_per_query * m ns; radius requests find 10 results per query)."""
import numpy as np
import pytest

from paper_1908_11807_amd import abx


def _server(**kw):
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
    # caller releases earlier ones
    s = _server(slots=4, budget_bytes=1 << 30, host_bytes=64 * 1024, sim_ns_per_query=100)
    q = np.zeros((200, 3), np.float32)
    tickets = [s.submit(0, abx.REQ_RADIUS, q, radius=0.1) for _ in range(20)]
    done = []
    for t in tickets:
        r = s.wait(t)
        assert r["status"] == abx.OK and r["total"] == 10 * 200
        # count and fill phases; a count that was sent back to the queue (its fill
        # waited on the others' host space) ran once more
        phases = r["t_device"] / (200 * 100e-9)
        assert phases == pytest.approx(round(phases)) and round(phases) >= 2
        done.append(r)
        s.release(t)
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
