"""Continuous-batching render server over a resident multi-level stack, admitted under an HBM
budget (memory-adaptive rendering: each request picks a level or a level range, section
Rendering Methods, and the server fits the work in flight to the memory it is given).

Structure
  BudgetLedger   bytes held on the device: the resident stack, every slot's workspace and the
                 frames in flight; allocations that would pass the budget are refused.
  Scheduler      arrival queue -> FIFO waiting queue -> slots. A request is admitted when a slot
                 is free and its estimated memory fits; requests that arrive while others are on
                 the GPU join as soon as a slot and memory free up (continuous batching). A request
                 whose allocation is refused mid-render is deferred with its exact need; one that
                 cannot fit even in an empty server is rejected.
  GpuExecutor    one libflod Renderer and one HIP stream per slot (slots' kernels overlap on the
                 device); workspace memory comes from torch's caching allocator through the
                 ledger, via the library's allocator callbacks.

Latency of a request = device completion - arrival (both host clock, seconds).
"""
from __future__ import annotations

import ctypes as C
import math
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


class WorkspaceRefused(Exception):
    """The render needed more memory than the ledger would give; `needed` is its total."""

    def __init__(self, needed: int):
        super().__init__(f"workspace refused, needs {needed} bytes")
        self.needed = int(needed)


class BudgetLedger:
    """Thread-safe byte ledger with a hard budget."""

    def __init__(self, budget: int, resident: int = 0):
        self.budget = int(budget)
        self.lock = threading.Lock()
        self.cond = threading.Condition(self.lock)
        self.held = int(resident)
        self.peak = self.held
        self.refusals = 0

    def try_take(self, nbytes: int) -> bool:
        with self.lock:
            if self.held + nbytes > self.budget:
                self.refusals += 1
                return False
            self.held += nbytes
            self.peak = max(self.peak, self.held)
            return True

    def give(self, nbytes: int) -> None:
        with self.cond:
            self.held -= int(nbytes)
            self.cond.notify_all()

    def free(self) -> int:
        with self.lock:
            return self.budget - self.held


@dataclass
class Completed:
    rid: int
    arrival: float
    admitted: float = math.nan
    done: float = math.nan
    status: str = "ok"          # ok | rejected | error
    slot: int = -1
    deferrals: int = 0
    result: object = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class _Job:
    req: object
    arrival: float
    reserve: int          # bytes the scheduler reserves for the request (its output frame)
    need: int             # bytes that must be free before it starts (exact after a deferral)
    deferrals: int = 0


class Scheduler:
    """FIFO admission of requests onto `n_slots` executor slots under a BudgetLedger.

    executor interface:
      estimate(req) -> bytes reserved for the request at admission (e.g. its output frame);
                       the executor charges its workspace to the ledger as it allocates
      run(slot, req) -> result; may raise WorkspaceRefused(needed)
      slot_bytes(slot) -> bytes the slot's workspace holds now
      trim(slot) -> free the slot's workspace
    """

    def __init__(self, executor, n_slots: int, ledger: BudgetLedger, keep_results: bool = False):
        self.ex = executor
        self.n_slots = int(n_slots)
        self.ledger = ledger
        self.keep_results = keep_results

    def serve(self, requests, time_scale: float = 1.0):
        """Replay `requests` (objects with .rid and .arrival_s) in real time; return the list of
        Completed records ordered by rid."""
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        out = {r.rid: Completed(r.rid, math.nan) for r in reqs}
        lock = threading.Condition()
        waiting: deque[_Job] = deque()
        free_slots = list(range(self.n_slots))
        busy = set()
        state = {"arrived": 0, "finished": 0, "stop": False}
        t0 = time.perf_counter()
        largest = self.ledger.budget - self.ledger.held   # room in an idle server

        def worker(slot: int, job: _Job, reserved: int):
            rec = out[job.req.rid]
            rec.admitted = time.perf_counter() - t0
            rec.slot = slot
            try:
                res = self.ex.run(slot, job.req)
                rec.done = time.perf_counter() - t0
                rec.status = "ok"
                rec.deferrals = job.deferrals
                if self.keep_results:
                    rec.result = res
                requeue = None
            except WorkspaceRefused as e:
                self.ex.trim(slot)
                job.deferrals += 1
                job.need = max(job.reserve, e.needed)
                requeue = job
            except Exception as e:  # pragma: no cover - reported, not swallowed
                rec.done = time.perf_counter() - t0
                rec.status = f"error: {e}"
                requeue = None
            self.ledger.give(reserved)
            with lock:
                busy.discard(slot)
                free_slots.append(slot)
                if requeue is not None:
                    if requeue.need > largest:
                        r2 = out[requeue.req.rid]
                        r2.status = "rejected"
                        r2.deferrals = requeue.deferrals
                        r2.done = time.perf_counter() - t0
                        state["finished"] += 1
                    else:
                        waiting.appendleft(requeue)
                else:
                    state["finished"] += 1
                lock.notify_all()

        def admit_locked():
            # FIFO: the head waits for memory rather than being overtaken
            while waiting and free_slots:
                job = waiting[0]
                if job.need > largest:
                    waiting.popleft()
                    rec = out[job.req.rid]
                    rec.status = "rejected"
                    rec.deferrals = job.deferrals
                    rec.done = time.perf_counter() - t0
                    state["finished"] += 1
                    continue
                slot = free_slots[-1]
                # the slot's own workspace is reused by the request, so it counts as free for it
                room = self.ledger.free() + self.ex.slot_bytes(slot)
                if room < job.need or not self.ledger.try_take(job.reserve):
                    # idle slots may hold workspace that the head needs: release it
                    for s in list(free_slots):
                        if self.ex.slot_bytes(s) > 0:
                            self.ex.trim(s)
                    room = self.ledger.free() + self.ex.slot_bytes(slot)
                    if room < job.need or not self.ledger.try_take(job.reserve):
                        return
                free_slots.pop()
                waiting.popleft()
                busy.add(slot)
                th = threading.Thread(target=worker, args=(slot, job, job.reserve), daemon=True)
                th.start()

        i = 0
        with lock:
            while state["finished"] < len(reqs):
                now = time.perf_counter() - t0
                while i < len(reqs) and reqs[i].arrival_s * time_scale <= now:
                    r = reqs[i]
                    out[r.rid].arrival = r.arrival_s * time_scale
                    est = int(self.ex.estimate(r))
                    waiting.append(_Job(r, r.arrival_s * time_scale, est, est))
                    i += 1
                admit_locked()
                if state["finished"] >= len(reqs):
                    break
                timeout = None
                if i < len(reqs):
                    timeout = max(0.0, reqs[i].arrival_s * time_scale - (time.perf_counter() - t0))
                lock.wait(timeout=timeout if timeout is not None else 0.05)
        return [out[r.rid] for r in sorted(reqs, key=lambda r: r.rid)]


def latency_stats(records) -> dict:
    ok = [r for r in records if r.status == "ok"]
    lat = np.array([r.latency for r in ok]) * 1e3
    span = max(r.done for r in ok) - min(r.arrival for r in ok) if ok else math.nan
    return {
        "completed": len(ok),
        "rejected": sum(r.status == "rejected" for r in records),
        "deferrals": int(sum(r.deferrals for r in records)),
        "p50_ms": float(np.percentile(lat, 50)) if ok else math.nan,
        "p99_ms": float(np.percentile(lat, 99)) if ok else math.nan,
        "mean_ms": float(lat.mean()) if ok else math.nan,
        "throughput_rps": len(ok) / span if ok else math.nan,
    }


# ---------------------------------------------------------------------------------------
# GPU executor
# ---------------------------------------------------------------------------------------

class GpuExecutor:
    """Renders requests over a resident stack; one Renderer and one HIP stream per slot.

    levels: list of render.GaussianLevel resident on the device (levels 1..L).
    d_proj: per-level band distances (d_proj[l-1] = d_proj^(l)); the centre of selection is
    each request's eye (per-view selection).
    """

    def __init__(self, levels, n_slots: int, ledger: BudgetLedger, d_proj, bg=(0.0, 0.0, 0.0), sh_degree=3,
                 keep_images: bool = False):
        import torch

        from . import _lib, render
        self.torch = torch
        self.render = render
        self._lib = _lib
        self.levels = levels
        self.ledger = ledger
        self.d_proj = list(d_proj)
        self.bg = bg
        self.sh_degree = sh_degree
        self.keep_images = keep_images
        self.device = levels[0].means.device
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_slots)]
        self.held = [0] * n_slots
        self._cbs = []
        self.renderers = []
        for s in range(n_slots):
            alloc, free = self._callbacks(s)
            self.renderers.append(render.Renderer(self.device.index, alloc=alloc, release=free))
        self.frame_bytes = {}

    def _callbacks(self, slot):
        torch = self.torch
        dev = self.device.index

        def alloc(user, nbytes, stream):
            if not self.ledger.try_take(int(nbytes)):
                return None
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), dev, self.streams[slot])
            except RuntimeError:
                self.ledger.give(int(nbytes))
                return None
            self.held[slot] += int(nbytes)
            return ptr

        def free(user, ptr, nbytes, stream):
            torch.cuda.caching_allocator_delete(ptr)
            self.held[slot] -= int(nbytes)
            self.ledger.give(int(nbytes))

        self._cbs.append((alloc, free))
        return alloc, free

    def slot_bytes(self, slot) -> int:
        return self.held[slot]

    def trim(self, slot) -> None:
        self.renderers[slot].trim(self.streams[slot])

    @staticmethod
    def frame_size(req) -> int:
        return 20 * int(req.camera.width) * int(req.camera.height)

    def estimate(self, req) -> int:
        """Bytes held by the request's output frame; the workspace is charged to the ledger as
        the library allocates it (the allocator refuses what would pass the budget)."""
        return self.frame_size(req)

    def run(self, slot, req):
        torch = self.torch
        r = self.renderers[slot]
        st = self.streams[slot]
        with torch.cuda.stream(st):
            try:
                if req.l_start == req.l_end:
                    img, T, nc = r.render_level(self.levels[req.l_start - 1], req.camera, self.bg,
                                                self.sh_degree, stream=st)
                else:
                    img, T, nc = r.render_selective(self.levels, req.l_start, req.l_end, self.d_proj,
                                                    req.camera.campos, req.camera, self.bg, self.sh_degree,
                                                    stream=st)
            except self._lib.FlodError as e:
                if e.status == self._lib.FLOD_ERR_WORKSPACE:
                    raise WorkspaceRefused(r.required_bytes() + self.frame_size(req)) from None
                raise
            st.synchronize()
        stats = r.stats()
        if self.keep_images:
            return {"image": img, "stats": stats}
        return {"stats": stats}


def serve_trace(levels, requests, n_slots=4, budget_bytes=32 << 30, d_proj=None, keep_images=False,
                time_scale=1.0):
    """Serve `requests` over the resident `levels` under `budget_bytes`; returns (records, stats)."""
    from . import synth
    resident = sum(lv.nbytes() for lv in levels)
    ledger = BudgetLedger(budget_bytes, resident)
    ex = GpuExecutor(levels, n_slots, ledger, d_proj if d_proj is not None else synth.LEVEL_BANDS,
                     keep_images=keep_images)
    sched = Scheduler(ex, n_slots, ledger, keep_results=keep_images)
    recs = sched.serve(requests, time_scale=time_scale)
    for s in range(n_slots):
        ex.trim(s)
    st = latency_stats(recs)
    st["peak_bytes"] = ledger.peak
    st["budget_bytes"] = budget_bytes
    st["resident_bytes"] = resident
    return recs, st
