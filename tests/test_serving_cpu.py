"""The continuous-batching scheduler on the CPU with a simulated executor (deterministic outputs,
service time a * sum(n^2) + b): admission, capacities, FIFO fairness, overlap of slots, per-event
results independent of the batch, and failure recovery."""
import threading
import time

import numpy as np
import pytest

from paper_2601_17554_amd.serve import CapacityError, Executor, Server, run_poisson


class FakeExecutor(Executor):
    def __init__(self, slots=2, max_rows=1000, max_events=4, a=2e-8, b=2e-3, fail_first=0,
                 always_fail=False, bytes_per_row=0, bytes_per_event=0, hbm_budget=None):
        self.max_rows, self.max_events, self._n = max_rows, max_events, slots
        self.bytes_per_row, self.bytes_per_event, self.hbm_budget = bytes_per_row, bytes_per_event, hbm_budget
        self.inflight, self.max_inflight = {}, 0
        self.a, self.b = a, b
        self.fail_first, self.always_fail = fail_first, always_fail
        self.batches, self.running, self.max_running = [], {}, 0
        self.lock = threading.Lock()

    def slots(self):
        return self._n

    def launch(self, slot, reqs):
        assert slot not in self.running
        assert len(reqs) <= self.max_events and sum(r.n for r in reqs) <= self.max_rows
        cost = self.a * sum(r.n ** 2 for r in reqs) + self.b
        self.running[slot] = time.perf_counter() + cost
        self.max_running = max(self.max_running, len(self.running))
        self.batches.append([r.n for r in reqs])
        self.inflight[slot] = self.footprint(sum(r.n for r in reqs), len(reqs))
        self.max_inflight = max(self.max_inflight, sum(self.inflight.values()))

    def done(self, slot):
        return time.perf_counter() >= self.running[slot]

    def footprint(self, rows, events):
        return rows * self.bytes_per_row + events * self.bytes_per_event

    def results(self, slot, reqs):
        del self.running[slot]
        self.inflight.pop(slot, None)
        if self.always_fail or self.fail_first > 0:
            self.fail_first -= 1
            raise RuntimeError("injected batch failure")
        return [{"logits": r.x[:, :6] * 2.0, "cls": np.argmax(r.x[:, :6], 1)} for r in reqs]

    def reset(self, slot):
        self.running.pop(slot, None)
        self.inflight.pop(slot, None)


def _events(count, seed=0, lo=1, hi=400):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((int(rng.integers(lo, hi)), 17)).astype(np.float32) for _ in range(count)]


def test_results_per_event_and_all_resolved():
    ex = FakeExecutor()
    srv = Server(ex)
    evs = _events(60)
    futs = [srv.submit(x) for x in evs]
    for x, f in zip(evs, futs):
        np.testing.assert_array_equal(f.result(timeout=10)["logits"], x[:, :6] * 2.0)
    srv.close()
    assert srv.stats["events"] == 60
    assert all(len(b) <= 4 and sum(b) <= 1000 for b in ex.batches)
    assert len(srv.latencies_ms()) == 60 and (srv.latencies_ms() > 0).all()


def test_slots_overlap_under_load():
    ex = FakeExecutor(slots=3, b=5e-3)
    srv = Server(ex)
    futs = [srv.submit(x) for x in _events(40, seed=1)]
    [f.result(timeout=10) for f in futs]
    srv.close()
    assert ex.max_running == 3 and srv.stats["max_inflight_slots"] == 3


def test_fifo_no_starvation_of_large_event():
    ex = FakeExecutor(slots=1, max_rows=1000, max_events=8)
    srv = Server(ex)
    small = _events(30, seed=2, lo=1, hi=50)
    futs = [srv.submit(x) for x in small[:10]]
    big = srv.submit(np.ones((990, 17), np.float32))
    futs += [srv.submit(x) for x in small[10:]]
    big.result(timeout=10)
    [f.result(timeout=10) for f in futs]
    srv.close()
    order = [n for b in ex.batches for n in b]
    assert order.index(990) <= 10  # admitted in arrival order: nothing that came later overtakes it


def test_capacity_rejected_at_submit():
    srv = Server(FakeExecutor(max_rows=1000))
    with pytest.raises(CapacityError):
        srv.submit(np.zeros((1001, 17), np.float32))
    with pytest.raises(ValueError):
        srv.submit(np.zeros((0, 17), np.float32))
    srv.close()


def test_failed_batch_is_retried_once():
    ex = FakeExecutor(fail_first=1)
    srv = Server(ex)
    futs = [srv.submit(x) for x in _events(8, seed=3)]
    [f.result(timeout=10) for f in futs]
    srv.close()
    assert srv.stats["failed_batches"] == 1 and srv.stats["events"] == 8


def test_persistent_failure_surfaces_to_caller():
    srv = Server(FakeExecutor(always_fail=True), retries=1)
    f = srv.submit(np.ones((5, 17), np.float32))
    with pytest.raises(RuntimeError, match="injected"):
        f.result(timeout=10)
    srv.close()


def test_poisson_driver():
    ex = FakeExecutor(slots=2, b=1e-3)
    srv = Server(ex)
    evs = _events(50, seed=4, hi=100)
    arrivals = np.cumsum(np.random.default_rng(5).exponential(1 / 2000.0, 50))
    wall = run_poisson(srv, evs, arrivals)
    srv.close()
    assert srv.stats["events"] == 50 and wall >= arrivals[-1]


def test_hbm_budget_binds_admission():
    """Admission by HBM footprint: with room for ~one 300-row batch in flight, three free slots
    still never hold more than the budget, admission waits for the budget, every event is served
    in FIFO order, and an event whose footprint alone exceeds the budget is refused at submit."""
    ex = FakeExecutor(slots=3, max_rows=1000, max_events=4, b=3e-3, bytes_per_row=1000,
                      bytes_per_event=5000, hbm_budget=320_000)
    srv = Server(ex)
    evs = [np.ones((n, 17), np.float32) * i for i, n in enumerate([150, 150, 100, 250, 60, 300, 90, 10] * 4)]
    futs = [srv.submit(x) for x in evs]
    for x, f in zip(evs, futs):
        np.testing.assert_array_equal(f.result(timeout=10)["logits"], x[:, :6] * 2.0)
    srv.close()
    assert ex.max_inflight <= 320_000 and srv.stats["max_inflight_bytes"] <= 320_000
    assert srv.stats["admission_blocked"] > 0
    assert ex.max_inflight > 150_000  # the budget, not a slot limit, is what bound the batches
    order = [n for b in ex.batches for n in b]
    assert order == [x.shape[0] for x in evs]
    assert len(srv.batch_log) == srv.stats["batches"] and all(b[2] <= 320_000 for b in srv.batch_log)
    with pytest.raises(CapacityError, match="budget"):
        srv2 = Server(FakeExecutor(bytes_per_row=1000, hbm_budget=100_000))
        try:
            srv2.submit(np.ones((200, 17), np.float32))
        finally:
            srv2.close()


def test_without_budget_slots_bound_only():
    ex = FakeExecutor(slots=3, b=3e-3, bytes_per_row=1000)
    srv = Server(ex)
    futs = [srv.submit(x) for x in _events(30, seed=6)]
    [f.result(timeout=10) for f in futs]
    srv.close()
    assert srv.stats["admission_blocked"] == 0 and ex.max_running == 3
