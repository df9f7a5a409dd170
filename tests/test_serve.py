"""Scheduling logic of the continuous-batching server, on the CPU: a mock
executor whose requests converge after a known number of iterations, and a
fake clock advanced by a step-cost model."""
import dataclasses

import numpy as np
import pytest

from paper_2111_14240_amd import serve


@dataclasses.dataclass
class MockProblem:
    bytes: int
    conv_iters: int
    work: float = 1.0


class MockExecutor:
    def __init__(self):
        self.active = {}          # rid -> [iters done, problem]
        self.admit_log = []
        self.max_bytes_seen = 0
        self.max_active_seen = 0

    def footprint(self, prob):
        return prob.bytes

    def work(self, prob):
        return prob.work

    def admit(self, req):
        self.active[req.rid] = [0, req.problem]
        self.admit_log.append(req.rid)
        self.max_large_seen = max(getattr(self, "max_large_seen", 0),
                                  sum(p.work >= 100 for _, p in self.active.values()))
        self.max_active_seen = max(self.max_active_seen, len(self.active))
        self.max_bytes_seen = max(self.max_bytes_seen, sum(p.bytes for _, p in self.active.values()))

    def step(self, n):
        for st in self.active.values():
            st[0] = min(st[0] + n, st[1].conv_iters)

    def poll(self):
        return {rid: (st[0] >= st[1].conv_iters, 0.01, st[0]) for rid, st in self.active.items()}

    def retire(self, rid):
        it, p = self.active.pop(rid)
        return ("x", rid, it)


def _requests(n=60, rate=20.0, seed=5):
    rng = np.random.default_rng(seed)
    arr = serve.poisson_arrivals(n, rate, seed)
    return [serve.Request(i, MockProblem(int(rng.integers(1, 9)) * 10**9, int(rng.integers(8, 60))),
                          float(arr[i])) for i in range(n)]


def step_cost(clock, n_active, iters):
    # one batched launch: a fixed cost plus a share per active request
    clock.advance(iters * (2e-3 + 0.5e-3 * n_active))


def test_poisson_arrivals_rate():
    a = serve.poisson_arrivals(20000, 20.0, 5)
    assert np.all(np.diff(a) > 0)
    assert abs(len(a) / a[-1] - 20.0) < 0.5


def test_all_requests_complete_with_memory_and_slot_limits():
    reqs = _requests()
    ex = MockExecutor()
    srv = serve.Server(ex, capacity_bytes=20 * 10**9, max_active=6, iters_per_step=4, on_step=step_cost)
    st = srv.run(reqs, serve.FakeClock())
    assert st.completed == len(reqs)
    assert ex.max_bytes_seen <= 20 * 10**9
    assert ex.max_active_seen <= 6
    for r in reqs:
        assert r.finished >= r.admitted >= r.arrival
        assert r.iters >= r.problem.conv_iters
        assert r.result == ("x", r.rid, r.problem.conv_iters)
    # FIFO admission
    assert ex.admit_log == sorted(ex.admit_log, key=lambda i: (reqs[i].arrival, i))
    assert st.p99 >= st.p50 > 0


def test_plain_runs_one_at_a_time_in_order():
    reqs = _requests(30)
    ex = MockExecutor()
    st = serve.run_plain(ex, reqs, serve.FakeClock(), on_step=step_cost)
    assert st.completed == 30 and st.max_active == 1
    fin = [r.finished for r in sorted(reqs, key=lambda r: r.arrival)]
    assert fin == sorted(fin)


def test_batching_beats_plain_under_load():
    """With a fixed per-launch cost, stepping many requests together finishes
    the same work sooner and with a shorter tail than one at a time."""
    a = _requests(80, rate=40.0)
    b = _requests(80, rate=40.0)
    served = serve.Server(MockExecutor(), 64 * 10**9, max_active=16, on_step=step_cost).run(
        a, serve.FakeClock())
    plain = serve.run_plain(MockExecutor(), b, serve.FakeClock(), on_step=step_cost)
    assert served.completed == plain.completed == 80
    assert served.p99 < plain.p99 and served.solves_per_s > plain.solves_per_s
    # equal work: every request ran exactly to its own convergence count
    assert [r.iters for r in a] == [r.iters for r in b]


def test_oversized_request_rejected():
    reqs = [serve.Request(0, MockProblem(10**12, 5), 0.0)]
    with pytest.raises(ValueError):
        serve.Server(MockExecutor(), capacity_bytes=10**9).run(reqs, serve.FakeClock())


def test_idle_gaps_wait_for_arrivals():
    reqs = [serve.Request(0, MockProblem(1, 4), 0.0), serve.Request(1, MockProblem(1, 4), 100.0)]
    clk = serve.FakeClock()
    st = serve.Server(MockExecutor(), 10, iters_per_step=4, on_step=step_cost).run(reqs, clk)
    assert st.completed == 2
    assert reqs[1].admitted >= 100.0


def test_size_classes_cap_large_requests_and_let_small_ones_pass():
    """At most max_large large requests are active; a small request that
    arrives while a large one waits for the large slot is admitted first."""
    reqs = [serve.Request(0, MockProblem(1, 40, work=500), 0.0),
            serve.Request(1, MockProblem(1, 40, work=500), 0.001),
            serve.Request(2, MockProblem(1, 8, work=1), 0.002),
            serve.Request(3, MockProblem(1, 8, work=1), 0.003)]
    ex = MockExecutor()
    srv = serve.Server(ex, capacity_bytes=100, max_active=8, iters_per_step=4, on_step=step_cost,
                       large_work=100, max_large=1)
    st = srv.run(reqs, serve.FakeClock())
    assert st.completed == 4 and ex.max_large_seen == 1
    assert ex.admit_log.index(2) < ex.admit_log.index(1)    # small passed the waiting large one
    assert reqs[1].admitted >= reqs[0].finished             # large ones run one after the other
    assert all(r.iters >= r.problem.conv_iters for r in reqs)


def test_size_classes_complete_a_random_mix():
    rng = np.random.default_rng(9)
    arr = serve.poisson_arrivals(120, 30.0, 9)
    reqs = [serve.Request(i, MockProblem(int(rng.integers(1, 5)) * 10**9, int(rng.integers(8, 80)),
                                         work=float(rng.choice([1, 10, 1000]))), float(arr[i]))
            for i in range(120)]
    ex = MockExecutor()
    st = serve.Server(ex, 20 * 10**9, max_active=12, on_step=step_cost, large_work=100,
                      max_large=2).run(reqs, serve.FakeClock())
    assert st.completed == 120 and ex.max_large_seen <= 2 and ex.max_active_seen <= 12
    assert ex.max_bytes_seen <= 20 * 10**9
