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

    def run(self, slot, req):
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
