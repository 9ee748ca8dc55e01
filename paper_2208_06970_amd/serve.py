"""Serving loop for decomposition jobs (one job = one volume through the whole
path: isobands and components, the Lloyd loop, statistics).

Requests arrive over time.  The scheduler admits them in arrival order into
a fixed number of slots (one HIP stream and one host thread each), as soon
as a slot is free and the job's device footprint fits the byte budget next
to the jobs in flight.  A job runs as a sequence of phases; at every phase
boundary of any job the scheduler releases what the finished phase needed
and re-examines the queue, so a request that arrives while others run joins
them as soon as memory and a slot free up (continuous batching at phase
granularity), and the admitted jobs overlap on the device.

Memory: a job reserves, on admission, its resident bytes (the outputs it
returns) plus the largest workspace of its remaining phases; each phase
allocates exactly its workspace as a fresh device tensor and frees it when
it ends, and after each phase the reservation shrinks to what the remaining
phases need.  So the device bytes in use never exceed the accounted bytes,
which never exceed the budget.  A request whose footprint alone exceeds the
budget is rejected at once; one that does not fit now waits (its admission
is deferred), also when an allocation of its phase fails on the device.

Failures and cancellation: a phase that raises fails its own request only
(its memory is released, the others continue); a queued request can be
cancelled (it is removed), a running one stops at its next phase boundary.

Every job computes exactly what it computes alone: the kernels and their
reduction orders do not depend on what else runs on the GPU.

The scheduling core (`Scheduler`) holds no threads and no clock: `serve`
drives it with host threads and wall time on the GPU, `simulate` with a
simulated clock and given phase durations (used by the CPU tests, with
phases that may fail and a budget that may refuse).
"""
from __future__ import annotations

import heapq
import threading
import time
from dataclasses import dataclass, field

import numpy as np

QUEUED, RUNNING, DONE, FAILED, CANCELLED, REJECTED = "queued", "running", "done", "failed", "cancelled", "rejected"


class DeferAdmission(Exception):
    """Raised by a phase whose device allocation failed: the request goes
    back to the head of the queue and is admitted again when memory frees."""


@dataclass
class Phase:
    name: str
    ws_bytes: int
    run: "object" = None   # run(request, workspace_tensor_or_None, stream) -> None (GPU runner only)


@dataclass
class Request:
    id: int
    job: "object"
    arrival: float
    resident_bytes: int
    phases: list
    status: str = QUEUED
    phase: int = 0                 # index of the running (or next) phase
    reserved: int = 0
    slot: int = -1
    start: float = float("nan")
    done: float = float("nan")
    error: "object" = None
    cancel_requested: bool = False
    defers: int = 0
    state: dict = field(default_factory=dict)   # outputs of finished phases

    def footprint(self, from_phase: int = 0) -> int:
        rest = self.phases[from_phase:]
        return int(self.resident_bytes + (max(p.ws_bytes for p in rest) if rest else 0))


class Budget:
    """Byte accounting against a fixed budget."""

    def __init__(self, budget_bytes: int):
        self.budget = int(budget_bytes)
        self.used = 0
        self.peak = 0

    def try_reserve(self, n: int) -> bool:
        if self.used + n > self.budget:
            return False
        self.used += n
        self.peak = max(self.peak, self.used)
        return True

    def release(self, n: int):
        self.used -= n
        assert self.used >= 0


class Scheduler:
    """Admission and phase bookkeeping (no threads, no clock).  Every method
    takes the current time; the runner calls them under one lock."""

    def __init__(self, slots: int, budget: Budget):
        self.budget = budget
        self.free_slots = list(range(slots))
        self.queue: list[Request] = []
        self.finished: list[Request] = []
        self.events: list[tuple] = []     # (time, what, request id) for reports and tests

    def submit(self, req: Request, now: float):
        req.arrival = now if req.arrival is None else req.arrival
        if req.footprint() > self.budget.budget:
            req.status = REJECTED
            req.done = now
            self.finished.append(req)
            self.events.append((now, "rejected", req.id))
            return
        self.queue.append(req)
        self.events.append((now, "queued", req.id))

    def cancel(self, req: Request, now: float):
        if req.status == QUEUED and req in self.queue:
            self.queue.remove(req)
            req.status = CANCELLED
            req.done = now
            self.finished.append(req)
            self.events.append((now, "cancelled", req.id))
        elif req.status == RUNNING:
            req.cancel_requested = True

    def admit(self, now: float) -> list:
        """Admit queued requests in arrival order while the head fits; returns
        the requests to start (their phase 0) with their slots."""
        started = []
        while self.queue and self.free_slots:
            req = self.queue[0]
            need = req.footprint(req.phase)
            if not self.budget.try_reserve(need):
                break                      # the head waits; arrival order is kept
            self.queue.pop(0)
            req.reserved = need
            req.slot = self.free_slots.pop(0)
            req.status = RUNNING
            if req.start != req.start:     # first admission
                req.start = now
            self.events.append((now, "admitted", req.id))
            started.append(req)
        return started

    def phase_done(self, req: Request, now: float, error=None) -> bool:
        """Book the end of req's current phase.  Returns True when req goes on
        with its next phase in the same slot, False when its slot is free
        again (finished, failed, cancelled or deferred)."""
        if isinstance(error, DeferAdmission):
            # the device could not allocate the phase's workspace: the job
            # drops what it produced and goes back to the head of the queue
            self._leave(req, now, QUEUED, "deferred")
            req.defers += 1
            req.phase = 0
            self.queue.insert(0, req)
            return False
        if error is not None:
            req.error = error
            self._leave(req, now, FAILED, "failed")
            return False
        req.phase += 1
        if req.phase >= len(req.phases):
            self._leave(req, now, DONE, "done")
            return False
        if req.cancel_requested:
            self._leave(req, now, CANCELLED, "cancelled")
            return False
        need = req.footprint(req.phase)   # only shrinks: the largest remaining workspace
        self.budget.release(req.reserved - need)
        req.reserved = need
        self.events.append((now, f"phase {req.phases[req.phase].name}", req.id))
        return True

    def _leave(self, req: Request, now: float, status: str, what: str):
        self.budget.release(req.reserved)
        req.reserved = 0
        self.free_slots.append(req.slot)
        self.free_slots.sort()
        req.slot = -1
        req.status = status
        if status != QUEUED:
            req.done = now
            self.finished.append(req)
        self.events.append((now, what, req.id))


# ---------------------------------------------------------------------------
# simulation (CPU): a simulated clock, given phase durations


def simulate(requests: list, slots: int, budget_bytes: int, duration, cancels=(), fail=None):
    """Run `requests` (arrival times set) through the scheduler on a simulated
    clock.  duration(request, phase) gives each phase's time; fail(request,
    phase, attempt) may return an exception to end that phase with;
    cancels = [(time, request id)].  Returns the scheduler."""
    sched = Scheduler(slots, Budget(budget_bytes))
    ev = []  # (time, order, kind, payload)
    order = 0

    def push(t, kind, payload):
        nonlocal order
        heapq.heappush(ev, (t, order, kind, payload))
        order += 1

    by_id = {r.id: r for r in requests}
    for r in requests:
        push(r.arrival, 0, r.id)           # kind 0: arrival
    for t, rid in cancels:
        push(t, 1, rid)                    # kind 1: cancel
    attempts = {}

    def start(req, now):
        k = (req.id, req.phase)
        attempts[k] = attempts.get(k, 0) + 1
        err = fail(req, req.phases[req.phase], attempts[k]) if fail else None
        push(now + duration(req, req.phases[req.phase]), 2, (req.id, err))   # kind 2: phase end

    while ev:
        now, _, kind, payload = heapq.heappop(ev)
        if kind == 0:
            sched.submit(by_id[payload], now)
        elif kind == 1:
            sched.cancel(by_id[payload], now)
        else:
            rid, err = payload
            req = by_id[rid]
            if sched.phase_done(req, now, err):
                start(req, now)
        for req in sched.admit(now):
            start(req, now)
    return sched


# ---------------------------------------------------------------------------
# GPU jobs


@dataclass
class Job:
    """Inputs of one job, already on the device."""
    field: "object"        # float32[nz, ny, nx]
    iso: "object"          # host float32[K]
    seeds: "object"        # int32[S] (uint32 bits)
    weights: "object"      # int16[nz, ny, nx] (uint16 bits) or None
    iters: int
    variables: "object"    # float32[m, nz, ny, nx]
    edges: "object" = None
    cov: bool = True
    cap_comp: int = 0      # bound on the component count (sizes the footprint)
    # results of the last serve() call (when kept)
    result: dict = field(default_factory=dict)
    arrival: float = 0.0
    start: float = 0.0
    done: float = 0.0
    status: str = ""

    @property
    def voxels(self) -> int:
        return int(self.field.numel())

    def _sizes(self):
        n = self.voxels
        S = int(self.seeds.numel())
        m = int(self.variables.shape[0])
        B = 0 if self.edges is None else int(self.edges.shape[1]) - 1
        nb = len(self.iso) + 1
        C = self.cap_comp or max(1024, n // 16)
        return n, S, m, B, nb, C

    def resident_bytes(self) -> int:
        """Device bytes of the outputs (labels, tables, statistics), rounded up
        for the allocator's 512-byte granularity."""
        n, S, m, B, nb, C = self._sizes()
        P = m * (m + 1) // 2
        labels = n * (1 + 4 + 4) + 4                  # band, comp, cell, status
        tables = C * (1 + 8 + 4) + (nb + 1) * 4 + S * 8
        per_cell = 8 + 4 * (4 * m + P) + 4 * m * B
        per_group = 8 + 8 * (2 * m + P) + 8 * m + 4 * m * B
        stats = S * per_cell + (C + nb) * per_group
        return int(labels + tables + stats + 64 * 512 + 3 * 256)

    def phases(self) -> list:
        from . import (lsrvt_aggregate_workspace_bytes, lsrvt_components_workspace_bytes,
                       lsrvt_cvt_workspace_bytes)
        n, S, m, B, nb, C = self._sizes()
        shape = tuple(self.field.shape)
        return [Phase("labels", lsrvt_components_workspace_bytes(shape, nb), _phase_labels),
                Phase("lloyd", lsrvt_cvt_workspace_bytes(shape, S, self.iters), _phase_lloyd),
                Phase("stats", lsrvt_aggregate_workspace_bytes(shape, S, C, nb, m, B, self.cov), _phase_stats)]

    def footprint(self) -> int:
        """Resident bytes plus the largest phase workspace."""
        return self.resident_bytes() + max(p.ws_bytes for p in self.phases())


class _OneShot:
    """A workspace that hands out one given device buffer (a phase's own,
    allocated with 256 bytes of slack for the alignment the library needs)."""

    def __init__(self, buf):
        self.buf = buf

    def get(self, nbytes):
        import ctypes
        nbytes = int(nbytes)
        if nbytes == 0:
            return None, 0
        base = 0 if self.buf is None else self.buf.data_ptr()
        off = (-base) % 256
        if self.buf is None or self.buf.numel() - off < nbytes:
            raise RuntimeError(f"phase workspace of {nbytes} bytes was not reserved")
        return ctypes.c_void_p(base + off), nbytes


def _phase_buffer(ws_bytes, device):
    import torch
    return torch.empty(ws_bytes + 256, dtype=torch.uint8, device=device) if ws_bytes else None


def _phase_labels(req, ws, stream):
    from . import lsrvt_components, lsrvt_isobands
    job = req.job
    band, status = lsrvt_isobands(job.field, job.iso, stream=stream)
    cc = lsrvt_components(band, len(job.iso) + 1, cap_comp=job.cap_comp or None, ws=_OneShot(ws), stream=stream)
    req.state.update(band=band, status=status, comp=cc)


def _phase_lloyd(req, ws, stream):
    from . import autotune, lsrvt_cvt
    job = req.job
    # the Voronoi schedule the autotuner found fastest for this job's class
    # (cached only: no measurement inside the serving loop)
    with autotune.engine_for(req.state["band"], job.seeds, len(job.iso) + 1, tune=False):
        r = lsrvt_cvt(req.state["band"], req.state["comp"].comp, job.seeds, job.weights, job.iters, ws=_OneShot(ws),
                      stream=stream, want_mean_ds=False)
    req.state["cvt"] = r


def _phase_stats(req, ws, stream):
    from . import lsrvt_aggregate
    job = req.job
    cc, r = req.state["comp"], req.state["cvt"]
    st = lsrvt_aggregate(r.cell, r.sites, r.site_comp, cc.comp_band, cc.n_comp, len(job.iso) + 1, job.variables,
                         job.edges, cov=job.cov, ws=_OneShot(ws), stream=stream)
    req.state["stats"] = st


def run_job(job: Job, ws=None, stream=None) -> dict:
    """The whole path for one job on `stream`, phases back to back."""
    import torch
    stream = stream or torch.cuda.current_stream()
    req = Request(0, job, 0.0, job.resident_bytes(), job.phases())
    with torch.cuda.stream(stream):
        for ph in req.phases:
            buf = _phase_buffer(ph.ws_bytes, job.field.device)
            ph.run(req, buf, stream)
            stream.synchronize()
            del buf
    return {"band": req.state["band"], "comp": req.state["comp"], "cvt": req.state["cvt"],
            "stats": req.state["stats"]}


@dataclass
class ServeReport:
    jobs: int
    slots: int
    budget_bytes: int
    makespan_s: float
    latencies_s: list
    voxel_iters: int
    peak_bytes: int                 # accounted (never above the budget)
    peak_device_bytes: int = 0      # torch.cuda.max_memory_allocated() above the start level
    statuses: dict = field(default_factory=dict)
    defers: int = 0

    def summary(self) -> dict:
        lat = np.asarray(self.latencies_s)
        return {"jobs": self.jobs, "slots": self.slots, "budget_gib": round(self.budget_bytes / 2**30, 2),
                "makespan_s": round(self.makespan_s, 4),
                "jobs_per_s": round(self.jobs / self.makespan_s, 3) if self.makespan_s else None,
                "gvox_iter_per_s": round(self.voxel_iters / self.makespan_s / 1e9, 4) if self.makespan_s else None,
                "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3) if len(lat) else None,
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3) if len(lat) else None,
                "mean_ms": round(float(lat.mean()) * 1e3, 3) if len(lat) else None,
                "peak_footprint_gib": round(self.peak_bytes / 2**30, 3),
                "peak_device_gib": round(self.peak_device_bytes / 2**30, 3),
                "statuses": self.statuses, "defers": self.defers}


def serve(jobs: list, arrivals: list, slots: int, budget_bytes: int, keep_results: bool = False,
          cancel_ids=()) -> ServeReport:
    """Run `jobs` arriving at `arrivals` (seconds from the start, nondecreasing)
    on `slots` streams under `budget_bytes` of device memory.  With
    `keep_results` the outputs of each finished job are handed to the caller
    (job.result) and from then on are the caller's memory, outside the
    budget; otherwise they are dropped when the job ends."""
    import torch
    if len(jobs) != len(arrivals):
        raise ValueError("one arrival time per job")
    device = jobs[0].field.device if jobs else None
    reqs = [Request(i, j, float(a), j.resident_bytes(), j.phases()) for i, (j, a) in enumerate(zip(jobs, arrivals))]
    if any(r.footprint() > budget_bytes for r in reqs):
        raise ValueError("a job alone exceeds the HBM budget")
    sched = Scheduler(slots, Budget(budget_bytes))
    lock = threading.Condition()
    work = {s: None for s in range(slots)}       # slot -> request to run next phase of
    stop = [False]
    streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
    torch.cuda.synchronize(device)
    base = torch.cuda.memory_allocated(device)
    torch.cuda.reset_peak_memory_stats(device)
    t0 = time.perf_counter()
    # inputs may have been written by work queued on the current stream
    ready = torch.cuda.current_stream(device).record_event()

    def worker(slot):
        st = streams[slot]
        st.wait_event(ready)
        while True:
            with lock:
                lock.wait_for(lambda: work[slot] is not None or stop[0])
                if work[slot] is None:
                    return
                req = work[slot]
            ph = req.phases[req.phase]
            err = None
            try:
                try:
                    buf = _phase_buffer(ph.ws_bytes, device)
                except torch.cuda.OutOfMemoryError as e:
                    raise DeferAdmission(str(e))
                with torch.cuda.stream(st):
                    ph.run(req, buf, st)
                st.synchronize()
                del buf
            except Exception as e:  # the request fails alone (or is deferred)
                err = e
            now = time.perf_counter() - t0
            with lock:
                go_on = sched.phase_done(req, now, err)
                if not go_on:
                    work[slot] = None
                    # a deferred job starts again from its first phase; the
                    # outputs of a finished job are handed over (kept) or dropped
                    if req.status != DONE or not keep_results:
                        if req.status == DONE:
                            req.state = {"_dropped": True}
                        else:
                            req.state.clear()
                for r in sched.admit(now):
                    work[r.slot] = r
                lock.notify_all()

    threads = [threading.Thread(target=worker, args=(s,), daemon=True) for s in range(slots)]
    for th in threads:
        th.start()
    cancel_ids = set(cancel_ids)
    for r in reqs:
        now = time.perf_counter() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        with lock:
            now = time.perf_counter() - t0
            sched.submit(r, r.arrival)
            if r.id in cancel_ids:
                sched.cancel(r, now)
            for q in sched.admit(now):
                work[q.slot] = q
            lock.notify_all()
    with lock:
        lock.wait_for(lambda: len(sched.finished) == len(reqs))
        stop[0] = True
        lock.notify_all()
    for th in threads:
        th.join()
    torch.cuda.synchronize(device)
    peak_dev = torch.cuda.max_memory_allocated(device) - base
    for r in reqs:
        j = r.job
        j.arrival, j.start, j.done, j.status = r.arrival, r.start, r.done, r.status
        j.result = ({"band": r.state["band"], "comp": r.state["comp"], "cvt": r.state["cvt"],
                     "stats": r.state["stats"]} if keep_results and r.status == DONE else {})
        r.state = {}
    failed = [r for r in reqs if r.status == FAILED]
    done = [r for r in reqs if r.status == DONE]
    makespan = (max(r.done for r in done) - min(r.arrival for r in done)) if done else 0.0
    lat = [r.done - r.arrival for r in done]
    vi = sum(r.job.voxels * max(r.job.iters, 1) for r in done)
    statuses = {}
    for r in reqs:
        statuses[r.status] = statuses.get(r.status, 0) + 1
    rep = ServeReport(len(done), slots, budget_bytes, makespan, lat, vi, sched.budget.peak, int(peak_dev), statuses,
                      sum(r.defers for r in reqs))
    rep.failed = [(r.id, r.error) for r in failed]
    return rep


def serial(jobs: list, arrivals: list) -> ServeReport:
    """The same request stream served one job at a time with plain launches
    (each job's calls back to back on one stream), for comparison."""
    import torch
    device = jobs[0].field.device if jobs else None
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    lat = []
    for j, a in zip(jobs, arrivals):
        now = time.perf_counter() - t0
        if a > now:
            time.sleep(a - now)
        run_job(j)
        lat.append(time.perf_counter() - t0 - a)
    makespan = (time.perf_counter() - t0 - min(arrivals)) if jobs else 0.0
    vi = sum(j.voxels * max(j.iters, 1) for j in jobs)
    return ServeReport(len(jobs), 1, 0, makespan, lat, vi, 0)


def poisson_arrivals(n: int, rate: float, seed: int) -> list:
    """n arrival times of a Poisson process of `rate` per second (seeded)."""
    rng = np.random.default_rng(seed)
    return list(np.cumsum(rng.exponential(1.0 / rate, size=n)))
