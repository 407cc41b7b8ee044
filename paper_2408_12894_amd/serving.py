"""Continuous-batching render server over a resident multi-level stack, admitted under an HBM
budget (memory-adaptive rendering: each request picks a level or a level range, section
Rendering Methods, and the server fits the work in flight to the memory it is given).

Structure
  BudgetLedger   bytes held against the budget; allocations that would pass it are refused.
                 DeviceLedger (the GPU executor's) charges what the device actually holds for
                 the process: torch's reserved bytes (the resident stack, slot workspaces,
                 frames and the blocks torch keeps cached after a free) plus the frames promised
                 to admitted requests, and admits an allocation only if it fits even when it
                 needs fresh memory of its full rounded size.
  Scheduler      arrival queue -> FIFO waiting queue -> slots. A request is admitted when a slot
                 is free and its estimated memory fits; requests that arrive while others are on
                 the GPU join as soon as a slot and memory free up (continuous batching). A request
                 whose allocation is refused mid-render is deferred with its exact need; one that
                 cannot fit even in an empty server is rejected, and so is a head that does not
                 fit when nothing is in flight and the server has released what it holds (memory
                 held outside it, such as results the caller keeps, then leaves no room that any
                 event could free). An executor may return a pending
                 result; one reaper thread completes those when their device work has finished.
  GpuExecutor    one libflod Renderer and one HIP stream per slot (slots' kernels overlap on the
                 device); workspace memory comes from torch's caching allocator through the
                 ledger, via the library's allocator callbacks. A request's work is bracketed by
                 two events on its slot stream: the device interval of every request, and the
                 completion the reaper polls (no thread blocks on a stream).

Latency of a request = completion - arrival (host clock, seconds); completion is when the
reaper sees the request's last event done.
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
        self.resident = int(resident)
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

    def room_when_idle(self) -> int:
        """Bytes an idle server can give a request (everything but the resident data)."""
        return self.budget - self.resident


def _torch_rounded(nbytes: int) -> int:
    """Bytes torch's caching allocator may newly reserve for one allocation of nbytes: under
    1 MiB from a 2 MiB segment, up to 10 MiB from a 20 MiB segment, beyond that rounded up to
    2 MiB."""
    n = int(nbytes)
    if n <= 1 << 20:
        return 2 << 20
    if n < 10 << 20:
        return 20 << 20
    return (n + (2 << 20) - 1) // (2 << 20) * (2 << 20)


class DeviceLedger(BudgetLedger):
    """A BudgetLedger whose held bytes are measured: torch's reserved bytes on the device plus
    the frame bytes promised to admitted requests. Since reserved memory includes what torch keeps
    cached after a free, a freed buffer counts until it is released (trim + empty_cache), and an
    allocation is allowed only if it fits when it needs fresh memory of its full rounded size:
    reserved + promised never passes the budget."""

    def __init__(self, budget: int, device):
        import torch
        self.torch = torch
        self.dev = device
        super().__init__(budget, 0)
        self.promised = 0
        self.idle_held = self._held()      # what an idle server holds (the resident stack)
        self.peak = self.idle_held

    def _held(self) -> int:
        return int(self.torch.cuda.memory_reserved(self.dev)) + self.promised

    def try_take(self, nbytes: int) -> bool:
        with self.lock:
            if self._held() + nbytes > self.budget:
                self.refusals += 1
                return False
            self.promised += int(nbytes)
            self.peak = max(self.peak, self._held())
            return True

    def give(self, nbytes: int) -> None:
        with self.cond:
            self.promised -= int(nbytes)
            self.cond.notify_all()

    def free(self) -> int:
        with self.lock:
            return self.budget - self._held()

    def room_when_idle(self) -> int:
        return self.budget - self.idle_held

    def allocate(self, nbytes: int, fn, promise: list | None = None):
        """fn() allocates nbytes (given as a list of its tensors' sizes or one size); run it if
        it fits and release the caller's promise (a one-element list, consumed) at the same
        time. Returns fn()'s result, or None when refused."""
        sizes = nbytes if isinstance(nbytes, (list, tuple)) else [nbytes]
        need = sum(_torch_rounded(n) for n in sizes)
        with self.lock:
            mine = promise[0] if promise else 0
            if self._held() - mine + need > self.budget:
                self.refusals += 1
                return None
            try:
                out = fn()
            except RuntimeError:
                return None
            if promise:
                self.promised -= promise[0]
                promise[0] = 0
            self.peak = max(self.peak, self._held())
            return out


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
    dev_start_ms: float = math.nan   # device interval on the slot stream (GPU executor)
    dev_end_ms: float = math.nan

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
    promise: list = field(default_factory=lambda: [0])   # reserve still held by the ledger


class Pending:
    """A request whose device work is enqueued; the reaper completes it when ready() is true."""

    def ready(self) -> bool:  # pragma: no cover - interface
        raise NotImplementedError

    def finish(self, rec: "Completed", keep: bool):  # pragma: no cover - interface
        """Fill the record from the finished work; return the result to keep (or None)."""
        raise NotImplementedError


class Scheduler:
    """FIFO admission of requests onto `n_slots` executor slots under a BudgetLedger.

    executor interface:
      estimate(req) -> bytes reserved for the request at admission (e.g. its output frame);
                       the executor charges its workspace to the ledger as it allocates
      run(slot, req, promise) -> result, or a Pending whose device work the reaper waits for;
                       may raise WorkspaceRefused(needed). promise is a one-element list holding
                       the admission reserve still charged; an executor that converts it into an
                       allocation sets it to 0 (the scheduler gives back what is left)
      slot_bytes(slot) -> bytes the slot's workspace holds now
      trim(slot) -> free the slot's workspace
    """

    def __init__(self, executor, n_slots: int, ledger: BudgetLedger, keep_results: bool = False):
        self.ex = executor
        self.n_slots = int(n_slots)
        self.ledger = ledger
        self.keep_results = keep_results

    def serve(self, requests, time_scale: float = 1.0):
        """Replay `requests` (objects with .rid and .arrival_s) in real time, arrival times scaled
        by time_scale (0: all at once); return the list of Completed records ordered by rid."""
        reqs = sorted(requests, key=lambda r: r.arrival_s)
        out = {r.rid: Completed(r.rid, math.nan) for r in reqs}
        lock = threading.Condition()
        waiting: deque[_Job] = deque()
        free_slots = list(range(self.n_slots))
        busy = set()
        pending = []                       # (slot, job, Pending) awaiting the reaper
        state = {"arrived": 0, "finished": 0, "stop": False}
        t0 = time.perf_counter()
        largest = self.ledger.room_when_idle()

        def release(slot: int, job: _Job, requeue) -> None:
            """Return the slot and what is left of the job's reserve; requeue or finish it."""
            self.ledger.give(job.promise[0])
            job.promise[0] = 0
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

        def worker(slot: int, job: _Job):
            rec = out[job.req.rid]
            rec.admitted = time.perf_counter() - t0
            rec.slot = slot
            requeue = None
            try:
                res = self.ex.run(slot, job.req, job.promise)
                if isinstance(res, Pending):
                    with lock:
                        pending.append((slot, job, res))
                        lock.notify_all()
                    return
                rec.done = time.perf_counter() - t0
                rec.status = "ok"
                rec.deferrals = job.deferrals
                if self.keep_results:
                    rec.result = res
            except WorkspaceRefused as e:
                self.ex.trim(slot)
                job.deferrals += 1
                job.need = max(job.reserve, e.needed)
                requeue = job
            except Exception as e:  # pragma: no cover - reported, not swallowed
                rec.done = time.perf_counter() - t0
                rec.status = f"error: {e}"
            release(slot, job, requeue)

        def reaper():
            while True:
                with lock:
                    if state["stop"] and not pending:
                        return
                    ready = [p for p in pending if p[2].ready()]
                    for p in ready:
                        pending.remove(p)
                    if not ready:
                        lock.wait(timeout=5e-5)
                        continue
                now = time.perf_counter() - t0
                for slot, job, res in ready:
                    rec = out[job.req.rid]
                    rec.done = now
                    rec.status = "ok"
                    rec.deferrals = job.deferrals
                    kept = res.finish(rec, self.keep_results)
                    if self.keep_results:
                        rec.result = kept
                    release(slot, job, None)

        rt = threading.Thread(target=reaper, daemon=True)
        rt.start()

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
                    # idle slots may hold workspace that the head needs, and memory freed by
                    # finished requests may still be cached: release both
                    for s_ in list(free_slots):
                        if self.ex.slot_bytes(s_) > 0:
                            self.ex.trim(s_)
                    release_cached = getattr(self.ex, "release_cached", None)
                    if release_cached is not None:
                        release_cached()
                    room = self.ledger.free() + self.ex.slot_bytes(slot)
                    if room < job.need or not self.ledger.try_take(job.reserve):
                        if busy:
                            return          # a request in flight will free memory
                        # nothing in flight, and what the server holds has been released: memory
                        # held outside it (results the caller keeps) leaves the head no room,
                        # and no event here will make room; waiting would never end
                        waiting.popleft()
                        rec = out[job.req.rid]
                        rec.status = "rejected"
                        rec.deferrals = job.deferrals
                        rec.done = time.perf_counter() - t0
                        state["finished"] += 1
                        continue
                job.promise[0] = job.reserve
                free_slots.pop()
                waiting.popleft()
                busy.add(slot)
                th = threading.Thread(target=worker, args=(slot, job), daemon=True)
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
            state["stop"] = True
            lock.notify_all()
        rt.join()
        return [out[r.rid] for r in sorted(reqs, key=lambda r: r.rid)]


def latency_stats(records) -> dict:
    ok = [r for r in records if r.status == "ok"]
    lat = np.array([r.latency for r in ok]) * 1e3
    span = max(r.done for r in ok) - min(r.arrival for r in ok) if ok else math.nan
    st = {
        "completed": len(ok),
        "rejected": sum(r.status == "rejected" for r in records),
        "deferrals": int(sum(r.deferrals for r in records)),
        "p50_ms": float(np.percentile(lat, 50)) if ok else math.nan,
        "p99_ms": float(np.percentile(lat, 99)) if ok else math.nan,
        "mean_ms": float(lat.mean()) if ok else math.nan,
        "throughput_rps": len(ok) / span if ok else math.nan,
    }
    st.update(device_overlap(ok))
    return st


def device_overlap(records) -> dict:
    """Overlap of the requests' device intervals (from the events on their slot streams):
    how many requests share device time with another, the union of the intervals (device busy
    with some request) against their sum, and the most requests in flight at once."""
    iv = sorted((r.dev_start_ms, r.dev_end_ms) for r in records
                if not (math.isnan(r.dev_start_ms) or math.isnan(r.dev_end_ms)))
    if not iv:
        return {}
    n = len(iv)
    overl = [False] * n
    reach, who = -math.inf, -1          # the furthest end among earlier intervals
    for k, (a, b) in enumerate(iv):
        if a < reach:
            overl[k] = True
            overl[who] = True
        if b > reach:
            reach, who = b, k
    ev = sorted([(a, 1) for a, _ in iv] + [(b, -1) for _, b in iv], key=lambda e: (e[0], e[1]))
    cur = best = 0
    union = 0.0
    last = None
    for t, d in ev:
        if cur > 0 and last is not None:
            union += t - last
        cur += d
        best = max(best, cur)
        last = t
    total = sum(b - a for a, b in iv)
    return {"device_requests": n, "device_overlapping": int(sum(overl)),
            "device_busy_ms": union, "device_sum_ms": total,
            "device_concurrency": total / union if union > 0 else math.nan, "device_max_in_flight": best}


# ---------------------------------------------------------------------------------------
# GPU executor
# ---------------------------------------------------------------------------------------

class _GpuPending(Pending):
    def __init__(self, ex, slot, ev0, ev1, frame, renderer):
        self.ex, self.slot, self.ev0, self.ev1, self.frame, self.r = ex, slot, ev0, ev1, frame, renderer

    def ready(self) -> bool:
        return self.ev1.query()

    def finish(self, rec, keep):
        rec.dev_start_ms = self.ex.t_ref.elapsed_time(self.ev0)
        rec.dev_end_ms = self.ex.t_ref.elapsed_time(self.ev1)
        stats = self.r.stats()
        res = {"image": self.frame[0], "stats": stats} if keep else None
        self.frame = None
        return res


class GpuExecutor:
    """Renders requests over a resident stack; one Renderer and one HIP stream per slot.

    levels: list of render.GaussianLevel resident on the device (levels 1..L).
    d_proj: per-level band distances (d_proj[l-1] = d_proj^(l)); the centre of selection is
    each request's eye (per-view selection).
    ledger: a DeviceLedger on the levels' device.
    """

    def __init__(self, levels, n_slots: int, ledger: DeviceLedger, d_proj, bg=(0.0, 0.0, 0.0), sh_degree=3):
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
        self.device = levels[0].means.device
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_slots)]
        self.held = [0] * n_slots
        self._cbs = []
        self.renderers = []
        for s in range(n_slots):
            alloc, free = self._callbacks(s)
            r = render.Renderer(self.device.index, alloc=alloc, release=free)
            r.keep_backward_state(False)   # the server only renders: no backward state in its workspace
            self.renderers.append(r)
        # device time reference for the requests' intervals
        self.t_ref = torch.cuda.Event(enable_timing=True)
        self.t_ref.record(torch.cuda.current_stream(self.device))
        self.t_ref.synchronize()

    def _callbacks(self, slot):
        torch = self.torch
        dev = self.device.index

        def alloc(user, nbytes, stream):
            ptr = self.ledger.allocate(
                int(nbytes), lambda: torch.cuda.caching_allocator_alloc(int(nbytes), dev, self.streams[slot]))
            if ptr is None:
                return None
            self.held[slot] += int(nbytes)
            return ptr

        def free(user, ptr, nbytes, stream):
            torch.cuda.caching_allocator_delete(ptr)
            self.held[slot] -= int(nbytes)

        self._cbs.append((alloc, free))
        return alloc, free

    def slot_bytes(self, slot) -> int:
        return self.held[slot]

    def trim(self, slot) -> None:
        """Release the slot's workspace back to the device (not only to torch's cache)."""
        self.renderers[slot].trim(self.streams[slot])
        self.release_cached()

    def release_cached(self) -> None:
        """Return the memory torch keeps cached (frames and workspace freed by finished
        requests) to the device."""
        self.torch.cuda.empty_cache()

    @staticmethod
    def frame_sizes(req):
        p = int(req.camera.width) * int(req.camera.height)
        return [12 * p, 4 * p, 4 * p]

    def estimate(self, req) -> int:
        """Bytes the request's output frame may reserve (rounded as torch reserves); the
        workspace is charged as the library allocates it (the ledger refuses what would pass
        the budget)."""
        return sum(_torch_rounded(n) for n in self.frame_sizes(req))

    def run(self, slot, req, promise=None):
        torch = self.torch
        r = self.renderers[slot]
        st = self.streams[slot]
        H, W = int(req.camera.height), int(req.camera.width)
        with torch.cuda.stream(st):
            frame = self.ledger.allocate(self.frame_sizes(req), lambda: (
                torch.empty((3, H, W), dtype=torch.float32, device=self.device),
                torch.empty((H, W), dtype=torch.float32, device=self.device),
                torch.empty((H, W), dtype=torch.int32, device=self.device)), promise)
            if frame is None:
                raise WorkspaceRefused(self.estimate(req) + r.workspace_bytes())
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(st)
            try:
                if req.l_start == req.l_end:
                    r.render_level(self.levels[req.l_start - 1], req.camera, self.bg, self.sh_degree, stream=st,
                                   out=frame)
                else:
                    r.render_selective(self.levels, req.l_start, req.l_end, self.d_proj, req.camera.campos,
                                       req.camera, self.bg, self.sh_degree, stream=st, out=frame)
            except self._lib.FlodError as e:
                if e.status == self._lib.FLOD_ERR_WORKSPACE:
                    raise WorkspaceRefused(r.required_bytes() + self.estimate(req)) from None
                raise
            ev1.record(st)
        return _GpuPending(self, slot, ev0, ev1, frame, r)


class Server:
    """A render server that stays up across traces: its slots' contexts keep their workspace
    (warm) between serve() calls. budget_bytes covers the resident stack and everything the
    server reserves on the device."""

    def __init__(self, levels, n_slots=4, budget_bytes=32 << 30, d_proj=None):
        import torch

        from . import synth
        self.torch = torch
        self.levels = levels
        self.n_slots = int(n_slots)
        self.budget = int(budget_bytes)
        self.dev = levels[0].means.device
        torch.cuda.synchronize(self.dev)
        torch.cuda.empty_cache()
        self.ledger = DeviceLedger(self.budget, self.dev)
        self.ex = GpuExecutor(levels, self.n_slots, self.ledger,
                              d_proj if d_proj is not None else synth.LEVEL_BANDS)

    def serve(self, requests, time_scale=1.0, keep_images=False):
        """Serve a trace; returns (records, stats), stats covering this call only."""
        torch = self.torch
        torch.cuda.synchronize(self.dev)
        torch.cuda.reset_peak_memory_stats(self.dev)
        self.ledger.peak = self.ledger._held()
        self.ledger.refusals = 0
        sched = Scheduler(self.ex, self.n_slots, self.ledger, keep_results=keep_images)
        recs = sched.serve(requests, time_scale=time_scale)
        torch.cuda.synchronize(self.dev)
        st = latency_stats(recs)
        st["peak_bytes"] = self.ledger.peak
        st["device_peak_reserved_bytes"] = int(torch.cuda.max_memory_reserved(self.dev))
        st["budget_bytes"] = self.budget
        st["resident_bytes"] = sum(lv.nbytes() for lv in self.levels)
        st["ledger_refusals"] = self.ledger.refusals
        return recs, st

    def close(self):
        for s in range(self.n_slots):
            self.ex.renderers[s].trim(self.ex.streams[s])
        self.torch.cuda.synchronize(self.dev)
        for rr in self.ex.renderers:
            rr.close()
        self.torch.cuda.empty_cache()


def serve_trace(levels, requests, n_slots=4, budget_bytes=32 << 30, d_proj=None, keep_images=False,
                time_scale=1.0):
    """Serve `requests` over the resident `levels` with a fresh server (cold contexts) under
    `budget_bytes`; returns (records, stats)."""
    srv = Server(levels, n_slots, budget_bytes, d_proj)
    try:
        return srv.serve(requests, time_scale=time_scale, keep_images=keep_images)
    finally:
        srv.close()
