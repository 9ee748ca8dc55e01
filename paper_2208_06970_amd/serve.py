"""Serving loop for decomposition jobs (one job = one volume through the whole
path: isobands, components, Lloyd loop, statistics).

Jobs arrive at given times.  A job is admitted, in arrival order, as soon as a
slot is free and its HBM footprint fits the budget next to the jobs already
running; each slot is a HIP stream driven by a host thread, so admitted jobs
overlap on the device (continuous batching at job granularity: a job that
arrives while others run starts as soon as a slot and memory free up, without
waiting for the running ones to finish).  Inputs stay resident on the device;
outputs are allocated per job.  Latency = completion - arrival.

Every job computes exactly what it computes alone: the kernels and their
reduction orders do not depend on what else runs on the GPU.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import (Workspace, lsrvt_aggregate, lsrvt_aggregate_workspace_bytes, lsrvt_components, lsrvt_cvt,
               lsrvt_cvt_workspace_bytes, lsrvt_isobands)


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
    # results
    result: dict = field(default_factory=dict)
    arrival: float = 0.0
    start: float = 0.0
    done: float = 0.0

    @property
    def voxels(self) -> int:
        return int(self.field.numel())

    def footprint(self) -> int:
        """Device bytes the job needs beyond its resident inputs: outputs and workspace."""
        n = self.voxels
        S = int(self.seeds.numel())
        m = int(self.variables.shape[0])
        B = 0 if self.edges is None else int(self.edges.shape[1]) - 1
        nb = len(self.iso) + 1
        C = self.cap_comp or max(1024, n // 16)
        P = m * (m + 1) // 2
        labels = n * (1 + 4 + 4)                      # band, comp, cell
        per_unit_cell = 8 + 4 * (4 * m + P) + 4 * m * B
        per_unit_group = 8 + 8 * (2 * m + P) + 8 * m + 4 * m * B
        stats = S * per_unit_cell + (C + nb) * per_unit_group
        tables = C * 13 + (nb + 1) * 4 + S * 8
        ws = max(lsrvt_cvt_workspace_bytes(self.field.shape, S, self.iters),
                 lsrvt_aggregate_workspace_bytes(self.field.shape, S, C, nb, m, B, self.cov))
        return int(labels + stats + tables + ws + (n // 64) * 4 * 8)


def run_job(job: Job, ws: Workspace, stream) -> dict:
    """The whole path for one job on `stream`; returns its outputs (tensors)."""
    import torch
    with torch.cuda.stream(stream):
        band, status = lsrvt_isobands(job.field, job.iso, stream=stream)
        cc = lsrvt_components(band, len(job.iso) + 1, cap_comp=job.cap_comp or None, ws=ws, stream=stream)
        r = lsrvt_cvt(band, cc.comp, job.seeds, job.weights, job.iters, ws=ws, stream=stream, want_mean_ds=False)
        st = lsrvt_aggregate(r.cell, r.sites, r.site_comp, cc.comp_band, cc.n_comp, len(job.iso) + 1, job.variables,
                             job.edges, cov=job.cov, ws=ws, stream=stream)
        stream.synchronize()
    return {"band": band, "comp": cc, "cvt": r, "stats": st}


@dataclass
class ServeReport:
    jobs: int
    slots: int
    budget_bytes: int
    makespan_s: float
    latencies_s: list
    voxel_iters: int
    peak_bytes: int

    def summary(self) -> dict:
        lat = np.asarray(self.latencies_s)
        return {"jobs": self.jobs, "slots": self.slots, "budget_gib": round(self.budget_bytes / 2**30, 2),
                "makespan_s": round(self.makespan_s, 4),
                "jobs_per_s": round(self.jobs / self.makespan_s, 3) if self.makespan_s else None,
                "gvox_iter_per_s": round(self.voxel_iters / self.makespan_s / 1e9, 4) if self.makespan_s else None,
                "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3) if len(lat) else None,
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3) if len(lat) else None,
                "mean_ms": round(float(lat.mean()) * 1e3, 3) if len(lat) else None,
                "peak_footprint_gib": round(self.peak_bytes / 2**30, 3)}


def serve(jobs: list, arrivals: list, slots: int, budget_bytes: int, keep_results: bool = False) -> ServeReport:
    """Run `jobs` arriving at `arrivals` (seconds from the start, nondecreasing) on `slots` streams."""
    import torch
    if len(jobs) != len(arrivals):
        raise ValueError("one arrival time per job")
    fps = [j.footprint() for j in jobs]
    if any(fp > budget_bytes for fp in fps):
        raise ValueError("a job alone exceeds the HBM budget")
    device = jobs[0].field.device if jobs else None
    cond = threading.Condition()
    free = list(range(slots))
    used = [0]
    peak = [0]
    streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
    wss = [Workspace(device) for _ in range(slots)]
    errors = []
    t0 = time.perf_counter()

    def worker(i: int, slot: int):
        job = jobs[i]
        try:
            job.start = time.perf_counter() - t0
            res = run_job(job, wss[slot], streams[slot])
            job.done = time.perf_counter() - t0
            if keep_results:
                job.result = res
        except Exception as e:  # reported after the loop
            errors.append((i, e))
        finally:
            with cond:
                used[0] -= fps[i]
                free.append(slot)
                cond.notify_all()

    threads = []
    for i, job in enumerate(jobs):
        job.arrival = float(arrivals[i])
        now = time.perf_counter() - t0
        if job.arrival > now:
            time.sleep(job.arrival - now)
        with cond:
            # arrival order: wait for a slot and room in the budget
            cond.wait_for(lambda: free and used[0] + fps[i] <= budget_bytes)
            slot = free.pop(0)
            used[0] += fps[i]
            peak[0] = max(peak[0], used[0])
        th = threading.Thread(target=worker, args=(i, slot))
        th.start()
        threads.append(th)
    for th in threads:
        th.join()
    if errors:
        raise RuntimeError(f"job {errors[0][0]} failed: {errors[0][1]}")
    makespan = max(j.done for j in jobs) - min(j.arrival for j in jobs) if jobs else 0.0
    lat = [j.done - j.arrival for j in jobs]
    vi = sum(j.voxels * max(j.iters, 1) for j in jobs)
    return ServeReport(len(jobs), slots, budget_bytes, makespan, lat, vi, peak[0])


def poisson_arrivals(n: int, rate: float, seed: int) -> list:
    """n arrival times of a Poisson process of `rate` per second (seeded)."""
    rng = np.random.default_rng(seed)
    return list(np.cumsum(rng.exponential(1.0 / rate, size=n)))
