"""Host-side tests of the request loop: admission by slot and footprint, FIFO order,
continuous admission while other solves run, error paths, latency statistics."""
import threading
import time

import numpy as np
import pytest

from paper_2302_09708_amd.serving import (AdmissionError, Request, Scheduler, nearest_rank, poisson_arrivals,
                                          summarize)


def _req(rid, arrival, fp, dur):
    r = Request(rid=rid, prob=None, ns=1, degree=1, n_iter=1, x_seed=0, arrival=arrival)
    r.fp, r.dur = fp, dur
    return r


class Fake:
    """open/run/close that sleep for a request's duration and log events."""

    def __init__(self):
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0
        self.events = []
        self.closed = []

    def open(self, req):
        return req, req.fp

    def run(self, req, slot):
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
            self.events.append(("start", req.rid, time.perf_counter()))
        time.sleep(req.dur)
        with self.lock:
            self.active -= 1
            self.events.append(("end", req.rid, time.perf_counter()))
        return req.rid * 10

    def close(self, req):
        self.closed.append(req.rid)


def test_nearest_rank_and_summary():
    v = [5, 1, 4, 2, 3, 10, 9, 8, 7, 6]
    assert nearest_rank(v, 50) == 5
    assert nearest_rank(v, 99) == 10
    assert nearest_rank(v, 10) == 1
    assert nearest_rank([3.0], 99) == 3.0
    with pytest.raises(ValueError):
        nearest_rank([], 50)


def test_poisson_arrivals_rate():
    a = poisson_arrivals(20000, 4.0, seed=5000)
    assert np.all(np.diff(a) > 0)
    assert abs(np.mean(np.diff(a)) - 0.25) < 0.01
    assert np.array_equal(a, poisson_arrivals(20000, 4.0, seed=5000))


def test_memory_admission_is_fifo_and_bounded():
    f = Fake()
    reqs = [_req(0, 0.0, 6, 0.15), _req(1, 0.0, 6, 0.05), _req(2, 0.0, 3, 0.05)]
    s = Scheduler(budget_bytes=10, slots=4, open_fn=f.open, run_fn=f.run, close_fn=f.close)
    res = s.run(reqs)
    assert [r.output for r in res] == [0, 10, 20]
    assert s.peak_bytes <= 10
    start = {rid: t for ev, rid, t in f.events if ev == "start"}
    end = {rid: t for ev, rid, t in f.events if ev == "end"}
    # request 1 does not fit beside request 0; request 2 fits but waits behind it (FIFO)
    assert start[1] >= end[0] - 1e-3
    assert start[2] >= start[1] - 1e-3
    assert sorted(f.closed) == [0, 1, 2]


def test_slots_bound_concurrency_and_overlap():
    f = Fake()
    reqs = [_req(i, 0.0, 1, 0.05) for i in range(6)]
    s = Scheduler(budget_bytes=1 << 30, slots=2, open_fn=f.open, run_fn=f.run, close_fn=f.close)
    s.run(reqs)
    assert f.max_active == 2 and s.peak_active == 2


def test_continuous_admission_while_others_run():
    f = Fake()
    # A runs long; B short; C arrives later and must start when B's slot frees, before A ends
    reqs = [_req(0, 0.0, 1, 0.5), _req(1, 0.0, 1, 0.05), _req(2, 0.02, 1, 0.05)]
    s = Scheduler(budget_bytes=100, slots=2, open_fn=f.open, run_fn=f.run, close_fn=f.close)
    res = s.run(reqs)
    start = {rid: t for ev, rid, t in f.events if ev == "start"}
    end = {rid: t for ev, rid, t in f.events if ev == "end"}
    assert end[1] - 1e-3 <= start[2] < end[0]
    assert res[2].latency < 0.3
    st = summarize(res)
    assert st["requests"] == 3 and st["p99_s"] >= st["p50_s"] > 0 and st["solves_per_s"] > 0


def test_oversize_request_is_refused():
    f = Fake()
    s = Scheduler(budget_bytes=10, slots=2, open_fn=f.open, run_fn=f.run, close_fn=f.close)
    with pytest.raises(AdmissionError):
        s.run([_req(0, 0.0, 11, 0.01)])
    assert f.closed == [0]


def test_worker_error_propagates_and_releases():
    f = Fake()

    def bad_run(req, slot):
        if req.rid == 1:
            raise RuntimeError("solve failed")
        return f.run(req, slot)

    s = Scheduler(budget_bytes=100, slots=2, open_fn=f.open, run_fn=bad_run, close_fn=f.close)
    with pytest.raises(RuntimeError, match="solve failed"):
        s.run([_req(0, 0.0, 1, 0.02), _req(1, 0.0, 1, 0.02), _req(2, 0.05, 1, 0.02)])
    assert 1 in f.closed


def test_failed_solve_is_reported_when_not_fail_fast():
    f = Fake()

    def bad_run(req, slot):
        if req.rid == 1:
            raise RuntimeError("solve failed")
        return f.run(req, slot)

    s = Scheduler(budget_bytes=100, slots=2, open_fn=f.open, run_fn=bad_run, close_fn=f.close, fail_fast=False)
    res = s.run([_req(0, 0.0, 1, 0.02), _req(1, 0.0, 1, 0.02), _req(2, 0.01, 1, 0.02)])
    assert [r.rid for r in res] == [0, 1, 2]
    assert res[1].error is not None and "solve failed" in res[1].error and res[1].output is None
    assert res[0].error is None and res[2].output == 20
    st = summarize(res)
    assert st["failed"] == 1 and st["requests"] == 3
    assert sorted(f.closed) == [0, 1, 2]


def test_bad_configuration():
    f = Fake()
    with pytest.raises(ValueError):
        Scheduler(budget_bytes=0, slots=1, open_fn=f.open, run_fn=f.run)
    with pytest.raises(ValueError):
        Scheduler(budget_bytes=10, slots=0, open_fn=f.open, run_fn=f.run)


def test_only_the_head_of_the_queue_is_opened():
    """Handles are created when a request reaches the head of the queue with a slot free:
    while the first request runs, the second waits opened (it does not fit beside it) and
    the third is not opened yet."""
    f = Fake()
    opened = []

    def open_log(req):
        opened.append((req.rid, time.perf_counter()))
        return f.open(req)

    reqs = [_req(0, 0.0, 6, 0.15), _req(1, 0.0, 6, 0.05), _req(2, 0.0, 3, 0.05)]
    s = Scheduler(budget_bytes=10, slots=4, open_fn=open_log, run_fn=f.run, close_fn=f.close)
    s.run(reqs)
    t_open = dict(opened)
    end = {rid: t for ev, rid, t in f.events if ev == "end"}
    assert [rid for rid, _ in opened] == [0, 1, 2]
    assert t_open[2] >= end[0] - 1e-3


def test_open_failure_joins_running_solves_and_closes():
    """An exception from open_fn ends the loop only after the admitted solves finish and
    are closed."""
    f = Fake()

    def bad_open(req):
        if req.rid == 1:
            raise RuntimeError("upload failed")
        return f.open(req)

    s = Scheduler(budget_bytes=100, slots=2, open_fn=bad_open, run_fn=f.run, close_fn=f.close)
    with pytest.raises(RuntimeError, match="upload failed"):
        s.run([_req(0, 0.0, 1, 0.1), _req(1, 0.01, 1, 0.01)])
    assert f.closed == [0] and f.active == 0
