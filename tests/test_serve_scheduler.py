"""The serving scheduler on the CPU: a mock device backend and a fake clock.

Covers admission by memory footprint, continuous batching over launch slots,
batch caps, failure isolation and re-queueing when a workspace was
under-estimated."""
import math

import numpy as np
import pytest

from paper_2412_00578_amd.serve import Request, Scheduler, WorkspaceTooSmall


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class MockBackend:
    """A batch of k requests takes fixed + per_item * k seconds of device time;
    batches on different slots run concurrently."""

    def __init__(self, clock, sizes, fixed=1e-3, per_item=0.5e-3, fail_rids=(),
                 undersized_rids=(), inflate=1.0):
        self.clock = clock
        self.sizes = sizes
        self.fixed, self.per_item = fixed, per_item
        self.fail_rids = set(fail_rids)
        self.undersized = dict.fromkeys(undersized_rids, 1)
        self.inflate = inflate
        self.launched = []
        self.max_inflight = 0
        self.inflight = 0

    def footprint(self, r):
        return self.sizes[r.scene]

    def launch(self, batch, slot):
        rids = {r.rid for r in batch}
        if rids & self.fail_rids:
            raise RuntimeError("injected launch error")
        for r in batch:
            if self.undersized.get(r.rid, 0) > 0:
                self.undersized[r.rid] -= 1
                raise WorkspaceTooSmall("pair count above the reservation")
        self.launched.append([r.rid for r in batch])
        self.inflight += 1
        self.max_inflight = max(self.max_inflight, self.inflight)
        return {"t_done": self.clock() + self.fixed + self.per_item * len(batch),
                "n": len(batch), "bytes": int(sum(self.sizes[r.scene] for r in batch) *
                                              self.inflate)}

    def bytes_in_flight(self, h):
        return h["bytes"]

    def done(self, h):
        return self.clock() >= h["t_done"]

    def wait(self, h):
        self.clock.t = max(self.clock.t, h["t_done"])

    def complete(self, h):
        self.inflight -= 1
        return [h["t_done"]] * h["n"]

    def release(self, h):
        pass


def _reqs(arrivals, scenes):
    return [Request(k, s, None, a) for k, (a, s) in enumerate(zip(arrivals, scenes))]


def _sched(backend, clock, pool=100, max_batch=4, slots=2):
    return Scheduler(backend, pool, max_batch, slots, clock=clock, sleep=clock.sleep)


def test_all_complete_fifo_and_latency_bounds():
    clock = FakeClock()
    be = MockBackend(clock, {0: 10, 1: 20})
    rng = np.random.default_rng(0)
    arr = np.cumsum(rng.exponential(1e-3, 200))
    reqs = _reqs(arr, rng.integers(0, 2, 200))
    st = _sched(be, clock).run(reqs)
    assert st.failed == 0 and all(r.status == "done" for r in reqs)
    order = [rid for b in be.launched for rid in b]
    assert order == sorted(order)                    # admitted in arrival order
    assert all(r.t_start >= r.arrival for r in reqs)
    assert all(r.t_done - r.t_start >= be.fixed + be.per_item - 1e-12 for r in reqs)
    assert st.pct(50) <= st.pct(99)


def test_memory_pool_bounds_batches():
    clock = FakeClock()
    be = MockBackend(clock, {0: 30})
    reqs = _reqs([0.0] * 40, [0] * 40)
    st = _sched(be, clock, pool=100, max_batch=8).run(reqs)
    assert st.peak_reserved_bytes <= 100
    assert max(len(b) for b in be.launched) <= 3     # 3 x 30 fits, 4 x 30 does not
    assert st.failed == 0


def test_oversized_request_runs_alone():
    clock = FakeClock()
    be = MockBackend(clock, {0: 10, 1: 500})
    reqs = _reqs([0.0, 0.0, 0.0, 0.0], [0, 1, 0, 0])
    st = _sched(be, clock, pool=100).run(reqs)
    assert st.failed == 0
    assert [1] in be.launched


def test_batches_overlap_on_two_slots_and_new_arrivals_join_next_batch():
    clock = FakeClock()
    be = MockBackend(clock, {0: 10}, fixed=5e-3, per_item=1e-3)
    # a first burst, then requests that arrive while it is on the device
    arr = [0.0] * 4 + [1e-3 * k for k in range(1, 9)]
    reqs = _reqs(arr, [0] * len(arr))
    st = _sched(be, clock, pool=1000, max_batch=4, slots=2).run(reqs)
    assert be.max_inflight == 2
    assert be.launched[0] == [0, 1, 2, 3]
    assert len(be.launched) >= 3 and st.failed == 0
    assert st.summary()["mean_batch"] > 1.0


def test_max_batch_respected():
    clock = FakeClock()
    be = MockBackend(clock, {0: 1})
    reqs = _reqs([0.0] * 50, [0] * 50)
    _sched(be, clock, pool=10**9, max_batch=5).run(reqs)
    assert max(len(b) for b in be.launched) == 5


def test_launch_error_fails_only_that_batch():
    clock = FakeClock()
    be = MockBackend(clock, {0: 10}, fail_rids={7})
    arr = [0.01 * k for k in range(20)]              # spaced: one request per batch
    reqs = _reqs(arr, [0] * 20)
    st = _sched(be, clock).run(reqs)
    assert st.failed == 1
    assert reqs[7].status == "failed" and "injected" in reqs[7].error
    assert all(r.status == "done" for r in reqs if r.rid != 7)
    assert len(st.latencies_ms) == 19


def test_undersized_workspace_is_requeued():
    clock = FakeClock()
    be = MockBackend(clock, {0: 10}, undersized_rids=[3, 4])
    reqs = _reqs([0.01 * k for k in range(10)], [0] * 10)
    st = _sched(be, clock).run(reqs)
    assert st.failed == 0 and st.requeued >= 2
    assert all(r.status == "done" for r in reqs)


def test_reservation_corrected_by_exact_bytes():
    # the backend reports twice its estimate once the pair count is known
    clock = FakeClock()
    be = MockBackend(clock, {0: 20}, inflate=2.0)
    reqs = _reqs([0.0] * 12, [0] * 12)
    st = _sched(be, clock, pool=100, max_batch=2, slots=3).run(reqs)
    assert st.failed == 0
    assert st.peak_reserved_bytes >= 80


def test_idle_server_sleeps_until_arrivals():
    clock = FakeClock()
    be = MockBackend(clock, {0: 1})
    reqs = _reqs([5.0, 10.0], [0, 0])
    st = _sched(be, clock).run(reqs)
    assert reqs[0].t_start >= 5.0 and reqs[1].t_start >= 10.0
    assert math.isclose(st.pct(50), 1.5, rel_tol=0.01)  # each alone: 1 ms + 0.5 ms


def test_warmup_arrivals_are_served_but_not_counted():
    clock = FakeClock()
    be = MockBackend(clock, {0: 10})
    arr = np.arange(60) * 2e-3
    reqs = _reqs(arr, [0] * 60)
    st = _sched(be, clock).run(reqs, skip=20)
    assert all(r.status == "done" for r in reqs)     # the warm-up is still served
    assert st.n == 40 and len(st.latencies_ms) == 40
    want = np.array([(r.t_done - r.arrival) * 1e3 for r in reqs[20:]])
    assert np.allclose(np.sort(st.latencies_ms), np.sort(want))
    assert st.wall_s == pytest.approx(max(r.t_done for r in reqs[20:]) - reqs[20].arrival)


def test_admission_bound_batches_are_counted():
    clock = FakeClock()
    be = MockBackend(clock, {0: 30})
    reqs = _reqs([0.0] * 12, [0] * 12)
    st = _sched(be, clock, pool=100, max_batch=8).run(reqs)
    # 3 x 30 fits, the 4th does not: every batch but the last closes on the pool
    assert st.admission_bound >= 1
    assert st.summary()["admission_bound_batches"] == st.admission_bound
    assert st.peak_reserved_bytes <= 100
