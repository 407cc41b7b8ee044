"""Serving scheduler on the CPU with a fake executor: admission under the HBM budget,
deferral of refused requests, rejection of requests that can never fit, FIFO order and
overlap of concurrent requests. Also the request-trace generator."""
import threading
import time
from dataclasses import dataclass

import numpy as np
import pytest

from paper_2408_12894_amd import serving, synth


@dataclass
class FakeReq:
    rid: int
    arrival_s: float
    work_s: float
    ws: int          # workspace bytes the render needs
    frame: int = 100


class FakeExecutor:
    """Sleeps for work_s; grows the slot's workspace through the ledger like libflod's
    grow-only buffers (refusal -> WorkspaceRefused with the exact total)."""

    def __init__(self, n_slots, ledger, under_estimate=False):
        self.ledger = ledger
        self.held = [0] * n_slots
        self.lock = threading.Lock()
        self.running = 0
        self.max_running = 0
        self.under = under_estimate

    def estimate(self, req):
        return req.frame

    def slot_bytes(self, slot):
        return self.held[slot]

    def trim(self, slot):
        if self.held[slot]:
            self.ledger.give(self.held[slot])
            self.held[slot] = 0

    def run(self, slot, req, promise=None):
        if self.held[slot] < req.ws:
            self.trim(slot)
            if not self.ledger.try_take(req.ws):
                raise serving.WorkspaceRefused(req.ws + req.frame)
            self.held[slot] = req.ws
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)
        time.sleep(req.work_s)
        with self.lock:
            self.running -= 1
        return {"rid": req.rid}


def serve(reqs, n_slots=4, budget=10_000, resident=1_000):
    ledger = serving.BudgetLedger(budget, resident)
    ex = FakeExecutor(n_slots, ledger)
    recs = serving.Scheduler(ex, n_slots, ledger).serve(reqs)
    return recs, ledger, ex


def test_all_complete_and_overlap():
    reqs = [FakeReq(i, 0.001 * i, 0.05, 500) for i in range(12)]
    recs, ledger, ex = serve(reqs)
    assert all(r.status == "ok" for r in recs)
    assert ex.max_running == 4                     # 4 slots busy at once
    assert ledger.peak <= ledger.budget
    for r in recs:
        assert r.admitted >= r.arrival - 1e-6 and r.done - r.admitted >= 0.05 - 1e-3
    st = serving.latency_stats(recs)
    assert st["completed"] == 12 and st["p99_ms"] >= st["p50_ms"] >= 50 - 1


def test_budget_serialises_large_requests():
    # each large request needs 4000 of the 9000 free bytes: at most two run at once
    reqs = [FakeReq(i, 0.0, 0.05, 4000) for i in range(6)]
    recs, ledger, ex = serve(reqs)
    assert all(r.status == "ok" for r in recs)
    assert ex.max_running <= 2
    assert ledger.peak <= ledger.budget


def test_oversized_request_is_rejected():
    reqs = [FakeReq(0, 0.0, 0.02, 500), FakeReq(1, 0.001, 0.02, 50_000), FakeReq(2, 0.002, 0.02, 500)]
    recs, ledger, ex = serve(reqs)
    assert [r.status for r in recs] == ["ok", "rejected", "ok"]
    assert recs[1].deferrals >= 1


def test_deferred_request_runs_when_memory_frees():
    # request 1 is refused while request 0 holds memory, then runs after it
    reqs = [FakeReq(0, 0.0, 0.15, 6000), FakeReq(1, 0.01, 0.02, 6000)]
    recs, ledger, ex = serve(reqs, n_slots=2)
    assert all(r.status == "ok" for r in recs)
    assert recs[1].done > recs[0].done
    assert recs[1].deferrals >= 1
    assert ledger.peak <= ledger.budget


def test_fifo_admission_order():
    reqs = [FakeReq(i, 0.0005 * i, 0.01, 100) for i in range(16)]
    recs, ledger, ex = serve(reqs, n_slots=2)
    adm = [r.admitted for r in sorted(recs, key=lambda r: r.arrival)]
    assert all(a <= b + 1e-6 for a, b in zip(adm, adm[1:]))


def test_idle_slot_workspace_is_released_for_the_head():
    # slot workspace from a finished request is trimmed when the next request needs the room
    reqs = [FakeReq(0, 0.0, 0.01, 5000), FakeReq(1, 0.05, 0.01, 300), FakeReq(2, 0.1, 0.01, 8000)]
    recs, ledger, ex = serve(reqs, n_slots=2)
    assert all(r.status == "ok" for r in recs)
    assert ledger.peak <= ledger.budget


def test_latency_stats():
    recs = [serving.Completed(i, arrival=0.0, admitted=0.0, done=(i + 1) * 0.001) for i in range(100)]
    st = serving.latency_stats(recs)
    assert abs(st["p50_ms"] - np.percentile(np.arange(1, 101), 50)) < 1e-9
    assert abs(st["p99_ms"] - np.percentile(np.arange(1, 101), 99)) < 1e-9


def test_trace_generator():
    tr = synth.serving_trace(seed=30, count=512)
    assert len(tr) == 512
    arr = np.array([r.arrival_s for r in tr])
    assert np.all(np.diff(arr) >= 0) and arr[0] == 0.0
    assert 0.0015 < np.diff(arr).mean() < 0.0025           # Poisson, mean gap 2 ms
    res = {(r.camera.width, r.camera.height) for r in tr}
    assert res <= set(synth.RESOLUTIONS) and len(res) == 4
    single = [r for r in tr if r.l_start == r.l_end]
    multi = [r for r in tr if r.l_start != r.l_end]
    assert 0.4 < len(single) / 512 < 0.6
    assert all((r.l_start, r.l_end) in synth.SELECTIVE_RANGES for r in multi)
    for r in tr[:20]:
        assert abs(np.linalg.norm(r.camera.campos) - 4.0) < 1e-5


class FakePending(serving.Pending):
    def __init__(self, t_start, work_s):
        self.t0, self.t1 = t_start, t_start + work_s

    def ready(self):
        return time.perf_counter() >= self.t1

    def finish(self, rec, keep):
        rec.dev_start_ms, rec.dev_end_ms = 1e3 * self.t0, 1e3 * self.t1
        return {"done_at": self.t1} if keep else None


class FakeAsyncExecutor(FakeExecutor):
    """Returns at once with a pending result that is ready work_s later (as the GPU executor
    returns once a request's work is enqueued): the scheduler's reaper completes it."""

    def run(self, slot, req, promise=None):
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)
        p = FakePending(time.perf_counter(), req.work_s)
        orig = p.finish

        def finish(rec, keep, _orig=orig):
            with self.lock:
                self.running -= 1
            return _orig(rec, keep)
        p.finish = finish
        return p


def test_pending_results_are_completed_by_the_reaper():
    reqs = [FakeReq(i, 0.001 * i, 0.03, 500) for i in range(12)]
    ledger = serving.BudgetLedger(10_000, 1_000)
    ex = FakeAsyncExecutor(4, ledger)
    recs = serving.Scheduler(ex, 4, ledger, keep_results=True).serve(reqs)
    assert all(r.status == "ok" for r in recs)
    assert ex.max_running == 4 and ex.running == 0
    for r in recs:
        assert r.done - r.admitted >= 0.03 - 1e-3 and r.result["done_at"] > 0
    st = serving.latency_stats(recs)
    assert st["completed"] == 12
    assert st["device_overlapping"] == 12 and st["device_max_in_flight"] == 4
    assert st["device_concurrency"] > 2.0
    assert ledger.held == 1_000 + sum(ex.held)      # every admission reserve was given back


def test_device_overlap_statistics():
    mk = lambda a, b: serving.Completed(0, 0.0, dev_start_ms=a, dev_end_ms=b)
    st = serving.device_overlap([mk(0, 10), mk(5, 15), mk(20, 30), mk(22, 24), mk(40, 41)])
    assert st["device_overlapping"] == 4 and st["device_max_in_flight"] == 2
    assert st["device_busy_ms"] == 26 and st["device_sum_ms"] == 33
    assert st["device_concurrency"] == 33 / 26
    assert serving.device_overlap([]) == {}


class FakeCachingExecutor(FakeExecutor):
    """Like a caching allocator: a finished request's frame stays charged (cached) until
    release_cached() returns it, so an idle server may hold memory that only a release frees."""

    def __init__(self, n_slots, ledger):
        super().__init__(n_slots, ledger)
        self.cached = 0
        self.releases = 0

    def run(self, slot, req, promise=None):
        out = super().run(slot, req, promise)
        with self.lock:
            if self.ledger.try_take(req.frame):   # the frame, cached after use
                self.cached += req.frame
        return out

    def release_cached(self):
        with self.lock:
            self.ledger.give(self.cached)
            self.cached = 0
            self.releases += 1


@pytest.mark.timeout(60)
def test_head_waits_for_cached_memory_to_be_released():
    """Memory held only in a cache must not stall the queue: when the head does not fit, the
    scheduler trims idle slots and releases the cache."""
    # one slot, workspace growing with every request: once a finished request's frame sits in
    # the cache, the next request's larger workspace fits only after the cache is released
    reqs = [FakeReq(i, 0.0005 * i, 0.005, 1500 + 100 * i, frame=600) for i in range(6)]
    ledger = serving.BudgetLedger(3_700, 1_000)
    ex = FakeCachingExecutor(1, ledger)
    recs = serving.Scheduler(ex, 1, ledger).serve(reqs)
    assert all(r.status == "ok" for r in recs)
    assert ex.releases > 0 and ledger.peak <= ledger.budget


class FakeKeepingExecutor(FakeExecutor):
    """A finished request's result keeps `keep` bytes on the device for as long as the caller
    holds it (the caller allocated it, so the budget check does not apply to it): memory that
    nothing inside the server will free."""

    def __init__(self, n_slots, ledger, keep):
        super().__init__(n_slots, ledger)
        self.keep = keep

    def run(self, slot, req, promise=None):
        out = super().run(slot, req, promise)
        with self.ledger.lock:
            self.ledger.held += self.keep
        return out


@pytest.mark.timeout(60)
def test_head_that_cannot_fit_with_nothing_in_flight_is_rejected():
    """Memory held outside the server can leave a deferred head no room even though it fit an
    idle server when serving began: with nothing in flight nothing will make room, so the head
    is rejected instead of waited for (waiting would never end)."""
    # budget 5000, resident 1000: 4000 for requests. Workspaces 1500, 2000, 2500, 3000, ... and
    # 600 kept per finished request: the fourth request's 3000 + 100 cannot fit beside the
    # 1800 kept, though it would fit an idle server
    reqs = [FakeReq(i, 0.001 * i, 0.002, 1500 + 500 * i, frame=100) for i in range(6)]
    ledger = serving.BudgetLedger(5_000, 1_000)
    ex = FakeKeepingExecutor(1, ledger, keep=600)
    recs = serving.Scheduler(ex, 1, ledger).serve(reqs)
    assert [r.status for r in recs[:3]] == ["ok", "ok", "ok"]
    assert all(r.status == "rejected" for r in recs[3:])
    assert recs[3].deferrals >= 1
