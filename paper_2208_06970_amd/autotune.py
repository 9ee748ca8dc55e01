"""Autotuner for the schedule choices of the hot path, with an on-disk cache.

Four choices are tuned by measurement on the GPU at hand (none of them
changes what is computed):

* the schedule of the Voronoi passes (``lsrvt_set_vt_engine``): the
  level-synchronous search or the brick relaxation.  Both give the same
  regions; which is faster depends on the volume's shape and how many voxels
  each site holds (wide cells mean many levels per pass but few relaxation
  rounds).  Tuned per job class by timing one Voronoi pass with each.
* the number of streams of ``lsrvt_batch_run``'s per-job phases (labels and
  statistics), tuned per batch by timing the whole batch;
* the launch shapes (``lsrvt_set_tuning``): the workgroups of a relaxation
  round (each walks the round's 16^3 bricks with that stride) and the tile
  the statistics stage in LDS per round (1, 2 or 4 voxels per thread), each
  tuned per job class by timing a short Lloyd loop (or one Voronoi pass)
  or one statistics call.

A job class is (GPU name, log2 of the voxel count, log2 of voxels per site,
band count bucket).  Results are kept in a JSON file (``LSRVT_AUTOTUNE_CACHE``,
by default ``~/.cache/lsrvt/autotune.json``), read once per process and
rewritten atomically (write to a temporary file, then rename) under a lock
file, so concurrent processes share it safely.  Nothing here changes what is
computed: every candidate gives bit-identical results.
"""
from __future__ import annotations

import json
import math
import os
import tempfile
import threading
import time

import numpy as np

from . import (TUNE_BR_GRID, TUNE_STATS_TILE, VT_BRICKS, VT_LEVELS, lsrvt_set_tuning, lsrvt_set_vt_engine,
               lsrvt_vt)

_LOCK = threading.Lock()
_CACHE = None


def cache_path() -> str:
    return os.environ.get("LSRVT_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "lsrvt", "autotune.json"))


def _device_name() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(torch.cuda.current_device()).name.replace(" ", "_")
    except Exception:  # pragma: no cover
        return "unknown"


def _load() -> dict:
    global _CACHE
    if _CACHE is None:
        try:
            with open(cache_path()) as fh:
                _CACHE = json.load(fh)
        except (OSError, ValueError):
            _CACHE = {}
    return _CACHE


def _store(key: str, value) -> None:
    """Record key -> value in memory and on disk (merged with what other
    processes wrote meanwhile)."""
    cache = _load()
    cache[key] = value
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        import fcntl
        with open(path + ".lock", "w") as lk:
            fcntl.flock(lk, fcntl.LOCK_EX)
            try:
                with open(path) as fh:
                    disk = json.load(fh)
            except (OSError, ValueError):
                disk = {}
            disk[key] = value
            fd, tmp = tempfile.mkstemp(dir=os.path.dirname(path), prefix=".autotune")
            with os.fdopen(fd, "w") as fh:
                json.dump(disk, fh, indent=1, sort_keys=True)
            os.replace(tmp, path)
            fcntl.flock(lk, fcntl.LOCK_UN)
    except OSError:  # a read-only home: keep the in-memory result
        pass


def job_class(shape, n_sites: int, n_bands: int) -> str:
    n = int(np.prod(shape))
    vps = n / max(int(n_sites), 1)
    return (f"vt:{_device_name()}:n2^{int(round(math.log2(max(n, 1))))}:"
            f"vps2^{int(round(math.log2(max(vps, 1.0))))}:bands{min(int(n_bands), 16)}")


def _time_vt(band, sites, engine: int, reps: int = 2) -> float:
    import torch
    prev = lsrvt_set_vt_engine(engine)
    try:
        lsrvt_vt(band, sites)  # warm-up (and workspace sizing)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            lsrvt_vt(band, sites)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps
    finally:
        lsrvt_set_vt_engine(prev)


def vt_engine(band, sites, n_bands: int, tune: bool = True) -> int | None:
    """The faster Voronoi schedule for this job's class: from the cache, or
    measured now (one pass with each schedule) when `tune`; None when the
    class is unknown and `tune` is False."""
    key = job_class(tuple(band.shape), int(sites.numel()), n_bands)
    with _LOCK:
        hit = _load().get(key)
    if hit is not None:
        return int(hit["engine"])
    if not tune:
        return None
    times = {e: _time_vt(band, sites, e) for e in (VT_LEVELS, VT_BRICKS)}
    best = min(times, key=times.get)
    with _LOCK:
        _store(key, {"engine": best, "ms": {str(k): round(v * 1e3, 4) for k, v in times.items()}})
    return best


class engine_for:
    """Context manager: run the enclosed calls of this thread with the tuned
    Voronoi schedule of the job (band, sites)."""

    def __init__(self, band, sites, n_bands: int, tune: bool = True):
        self.engine = vt_engine(band, sites, n_bands, tune)
        self.prev = None

    def __enter__(self):
        if self.engine is not None:
            self.prev = lsrvt_set_vt_engine(self.engine)
        return self

    def __exit__(self, *exc):
        if self.prev is not None:
            lsrvt_set_vt_engine(self.prev)
        return False


def batch_streams(make_jobs, candidates=(2, 4, 8), key: str | None = None, ws=None) -> int:
    """The number of streams for lsrvt_batch_run: cached under `key`, or
    measured by running the batch (make_jobs() -> list of BatchJob) with each
    candidate."""
    import torch
    from . import lsrvt_batch_run
    if key is not None:
        with _LOCK:
            hit = _load().get(f"batch:{_device_name()}:{key}")
        if hit is not None:
            return int(hit["streams"])
    times = {}
    for n in candidates:
        lsrvt_batch_run(make_jobs(), n_streams=n, ws=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lsrvt_batch_run(make_jobs(), n_streams=n, ws=ws)
        torch.cuda.synchronize()
        times[n] = time.perf_counter() - t0
    best = min(times, key=times.get)
    if key is not None:
        with _LOCK:
            _store(f"batch:{_device_name()}:{key}", {"streams": best,
                                                     "ms": {str(k): round(v * 1e3, 3) for k, v in times.items()}})
    return best


def _cached(key):
    with _LOCK:
        return _load().get(key)


def _time(fn, reps: int = 2) -> float:
    import torch
    fn()  # warm-up (and workspace sizing)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def br_grid(band, sites, n_bands: int, candidates=(1024, 2048, 4096, 8192), tune: bool = True, comp=None,
            weights=None, iters: int = 2) -> int | None:
    """Workgroups per relaxation round for this job class: cached, or
    measured now with each candidate by brick relaxation — a short Lloyd
    loop (`iters` updates: one full pass, then incremental ones, which
    dominate a long loop) when the components `comp` are given, else one
    Voronoi pass."""
    key = "brgrid:" + job_class(tuple(band.shape), int(sites.numel()), n_bands)
    hit = _cached(key)
    if hit is not None:
        return int(hit["grid"])
    if not tune:
        return None
    from . import lsrvt_cvt
    if comp is not None:
        def run():
            lsrvt_cvt(band, comp, sites, weights, iters, want_mean_ds=False)
    else:
        def run():
            lsrvt_vt(band, sites)
    prev_e = lsrvt_set_vt_engine(VT_BRICKS)
    times = {}
    try:
        for gsz in candidates:
            prev = lsrvt_set_tuning(TUNE_BR_GRID, gsz)
            try:
                times[gsz] = _time(run)
            finally:
                lsrvt_set_tuning(TUNE_BR_GRID, prev)
    finally:
        lsrvt_set_vt_engine(prev_e)
    best = min(times, key=times.get)
    with _LOCK:
        _store(key, {"grid": best, "ms": {str(k): round(v * 1e3, 4) for k, v in times.items()}})
    return best


def stats_tile(shape, n_sites: int, n_bands: int, n_vars: int, run, candidates=(1, 2, 4),
               tune: bool = True) -> int | None:
    """Voxels per thread and staging round of the statistics for this job
    class (shape, sites, bands, variable count): cached, or measured now by
    timing run() (one lsrvt_aggregate call) with each."""
    key = f"statstile:m{int(n_vars)}:" + job_class(tuple(shape), int(n_sites), n_bands)
    hit = _cached(key)
    if hit is not None:
        return int(hit["tile"])
    if not tune:
        return None
    times = {}
    for v in candidates:
        prev = lsrvt_set_tuning(TUNE_STATS_TILE, v)
        try:
            times[v] = _time(run)
        finally:
            lsrvt_set_tuning(TUNE_STATS_TILE, prev)
    best = min(times, key=times.get)
    with _LOCK:
        _store(key, {"tile": best, "ms": {str(k): round(v * 1e3, 4) for k, v in times.items()}})
    return best


class shapes:
    """Context manager: run the enclosed calls of this thread with the given
    launch shapes (None leaves a knob at the library's choice)."""

    def __init__(self, br_grid: int | None = None, stats_tile: int | None = None):
        self.want = {TUNE_BR_GRID: br_grid, TUNE_STATS_TILE: stats_tile}
        self.prev = {}

    def __enter__(self):
        for k, v in self.want.items():
            if v is not None:
                self.prev[k] = lsrvt_set_tuning(k, v)
        return self

    def __exit__(self, *exc):
        for k, v in self.prev.items():
            lsrvt_set_tuning(k, v)
        return False
