"""Benchmark of the level-set restricted Voronoi hot path on one MI355X.

One step = the whole hot path over one synthetic volume, with all inputs
already resident in HBM: isobands -> components -> Lloyd loop (T updates and
T + 1 restricted geodesic Voronoi passes) -> statistics of every cell merged to
components and bands.  The initial sites are an input of the Lloyd loop; they
are drawn once before timing from the (deterministic) components.

Default workload (the largest configuration that fits one GPU): the
combustion-shaped 1024 x 512 x 512 volume, a thin wrinkled flame sheet
standing in for the paper's DNS flame data (10 isovalues of the mixture
fraction Z, |grad T| saliency weights as uint16, one site per 4096
weight-scaled voxels, 30 updates, 18 statistics variables (Z, T, 16 species)
with 32-bin histograms and the full 18 x 18 covariance).

value = voxels * T / step time, in Gvoxels/s per Lloyd iteration, with the
whole step (isobands, components, final pass and statistics included) in the
denominator.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extras]
                       [--fourier | --batch | --serve]

The main line also carries, as extra keys, the 256^3 Fourier workload's step
("fourier256"), the 64-volume batch through lsrvt_batch_run against one job
at a time ("batch") and a short Poisson serving run against serial plain
launches ("serve"), unless --no-extras.

Modes that print their own JSON line instead of the main one:
  --fourier the 256^3 Fourier workload (8 isovalues, |grad f| weights, 20
            updates, 8 variables), with the joint moments, on-device seeding
            and line-of-sight Lloyd loop timed beside it;
  --batch   64 independent Fourier volumes (edges 32..192, cubes and 2:1:1
            boxes, 3..10 isovalues, 15 updates) through lsrvt_batch_run,
            against the same jobs run one at a time;
  --serve   a Poisson stream of jobs of the serving configuration's sizes
            (edges 64..512 per axis, 3..12 isovalues, 10..30 updates, 4..16
            variables) through the serving loop with HBM-footprint admission,
            against serial plain launches; p50/p99 latency and throughput per
            arrival rate.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
VT_BYTES_PER_VOXEL = 5           # one Voronoi pass must read the band (1 B) and write the cell (4 B)
LOS_BYTES_PER_VOXEL = 20         # a line-of-sight pass: comp in (4 B); length, source, cell out (8 + 4 + 4 B)
PROFILES = os.path.join(ROOT, "profiles")
CVT_SOURCE = os.path.join(ROOT, "paper_2208_06970_amd", "csrc", "cvt.hip")


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _source_hash():
    with open(CVT_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic_per_launch(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary, or None when it is missing or the kernel
    source changed since the counters were taken."""
    try:
        with open(os.path.join(PROFILES, f"{kernel}_traffic_{workload}.json")) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256_16") != _source_hash():
        return None
    return rec.get("bytes_per_launch")


def _host_cpu():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return model


def cpu_baseline(field, iso, weights, variables, edges, rho, seed, iters, sample_desc, T_sample=2):
    """The oracle as it stands, single-threaded, on a bounded sample: every
    phase timed on its own (isobands, components, T_sample + 1 Voronoi passes,
    T_sample updates, three levels of statistics), the per-voxel rate of a
    step with `iters` updates formed from the per-phase times (the fixed
    phases counted once, the Voronoi pass iters + 1 times and the update iters
    times, as in the GPU step)."""
    import numpy as np
    import oracle
    import synth
    t = {}
    t0 = time.perf_counter()
    band = oracle.bands(field, iso)
    t["isobands"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    cc = oracle.components(band, len(iso) + 1)
    t["components"] = time.perf_counter() - t0
    sites = synth.flame_sites(cc.comp, cc.n_comp, weights, rho, seed)
    t_vt, t_up = [], []
    s = sites.copy()
    for k in range(T_sample + 1):
        t0 = time.perf_counter()
        cell = oracle.vt(cc.comp, s)
        t_vt.append(time.perf_counter() - t0)
        if k == T_sample:
            break
        t0 = time.perf_counter()
        s, _ = oracle.update(cell, s, weights)
        t_up.append(time.perf_counter() - t0)
    S = len(sites)
    site_comp = cc.comp.ravel()[sites]
    t0 = time.perf_counter()
    oracle.stats(cell, S, variables, edges, cov=True)
    cu = np.where(cell == oracle.NONE_ID, oracle.NONE_ID, site_comp[np.minimum(cell, S - 1)]).astype(np.uint32)
    oracle.stats(cu, cc.n_comp, variables, edges, cov=True)
    bu = np.where(cell == oracle.NONE_ID, oracle.NONE_ID, band.astype(np.uint32))
    oracle.stats(bu, len(iso) + 1, variables, edges, cov=True)
    t["statistics"] = time.perf_counter() - t0
    t["vt_pass"] = float(np.mean(t_vt))
    t["update"] = float(np.mean(t_up))
    step = t["isobands"] + t["components"] + (iters + 1) * t["vt_pass"] + iters * t["update"] + t["statistics"]
    n = field.size
    return {"value": n * iters / step / 1e9, "unit": "Gvoxels/s per Lloyd iteration", "cores": 1, "kind": "oracle",
            "seconds": round(sum(v for k, v in t.items() if k not in ("vt_pass", "update")) + sum(t_vt) + sum(t_up), 3),
            "phase_seconds": {k: round(v, 4) for k, v in t.items()},
            "lloyd_iter_gvox_s": round(n / (t["vt_pass"] + t["update"]) / 1e9, 6),
            "host_cpu": _host_cpu(), "host_threads": len(os.sched_getaffinity(0)),
            "sample": sample_desc + f"; {T_sample} updates timed per phase, the step formed for T={iters}; "
                                    "single-threaded C"}


class Step:
    """One whole step of the hot path on device-resident inputs, with
    per-phase hipEvent timing."""

    def __init__(self, f, iso, n_bands, sd, w, iters, x, e):
        import torch
        self.f, self.iso, self.n_bands, self.sd, self.w, self.iters, self.x, self.e = f, iso, n_bands, sd, w, iters, x, e
        self.ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        self.ph = [0.0] * 4
        self.n = 0

    def __call__(self, record):
        import torch
        import paper_2208_06970_amd as L
        if record:
            self.ev[0].record()
        b, _ = L.lsrvt_isobands(self.f, self.iso)
        if record:
            self.ev[1].record()
        c = L.lsrvt_components(b, self.n_bands)
        if record:
            self.ev[2].record()
        r = L.lsrvt_cvt(b, c.comp, self.sd, self.w, self.iters, want_mean_ds=False)
        if record:
            self.ev[3].record()
        L.lsrvt_aggregate(r.cell, r.sites, r.site_comp, c.comp_band, c.n_comp, self.n_bands, self.x, self.e, cov=True)
        if record:
            self.ev[4].record()
            torch.cuda.synchronize()
            for k in range(4):
                self.ph[k] += self.ev[k].elapsed_time(self.ev[k + 1])
            self.n += 1
        return r, c

    def phases(self):
        return {k: round(v / max(self.n, 1), 4) for k, v in zip(("isobands", "components", "lloyd", "aggregate"),
                                                                 self.ph)}


def timed_steps(step, steps, warmup, label):
    """Warm-up, then exactly `steps` timed steps bracketed by synchronisations;
    also the Voronoi level kernel's own time (hipEvents on its stream)."""
    import torch
    import paper_2208_06970_amd as L
    for i in range(warmup):
        step(False)
        _log(f"{label}: warmup {i + 1}/{warmup} done")
    torch.cuda.synchronize()
    L.lsrvt_timing_read()                      # discard anything recorded so far
    L.lsrvt_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(True)
        _log(f"{label}: step {i + 1}/{steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    L.lsrvt_timing_enable(False)
    return dt * 1e3 / steps, L.lsrvt_timing_read()


def roofline(timing, workload):
    """Roofline of the Voronoi passes' dominant kernel, from the library's own
    hipEvent brackets: the level kernel (one launch per BFS level) or the
    relaxation round (one brick-list launch and one round launch per round).
    Algorithmic bytes of one pass: read the band, write the cell (5 B per
    voxel), spread over the pass's launches."""
    vt_ms, vt_launches, vt_passes, vox_per_pass, engines = timing
    kernel = {1: "k_bfs_level", 2: "k_br_round"}.get(engines, "k_bfs_level+k_br_round")
    alg_bytes_per_launch = VT_BYTES_PER_VOXEL * vox_per_pass * vt_passes / max(vt_launches, 1)
    avg_launch_s = vt_ms / 1e3 / max(vt_launches, 1)
    achieved = alg_bytes_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    return {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": _traffic_per_launch(kernel, workload),
            "avg_launch_us": round(avg_launch_s * 1e6, 3), "launches": vt_launches, "passes": vt_passes,
            "alg_bytes_per_launch": round(alg_bytes_per_launch, 1),
            "pass_ms": round(vt_ms / max(vt_passes, 1), 3)}


def bench_flame(args):
    """The main line: the whole step on the combustion-shaped 1024 x 512 x 512 volume."""
    import numpy as np
    import torch
    import paper_2208_06970_amd as L
    import synth
    _log("flame: generating the 1024x512x512 workload")
    wl = synth.flame_workload()
    n = wl.field.size
    f = torch.from_numpy(wl.field).cuda()
    w = torch.from_numpy(wl.weights.view(np.int16)).cuda()
    x = torch.from_numpy(np.ascontiguousarray(wl.variables)).cuda()
    e = torch.from_numpy(wl.edges).cuda()
    band, _ = L.lsrvt_isobands(f, wl.iso)
    cc = L.lsrvt_components(band, wl.n_bands)
    seeds = synth.flame_sites(cc.comp.cpu().numpy().view(np.uint32), cc.n_comp, wl.weights, wl.rho, wl.seed)
    sd = torch.from_numpy(seeds.view(np.int32)).cuda()
    _log(f"flame: comps={cc.n_comp} sites={len(seeds)}")
    step = Step(f, wl.iso, wl.n_bands, sd, w, wl.iters, x, e)
    # launch shapes for this job class, tuned before timing (cached on disk)
    from paper_2208_06970_amd import autotune
    _log("flame: tuning launch shapes")
    grid = autotune.br_grid(band, sd, wl.n_bands, comp=cc.comp, weights=w)
    r1 = L.lsrvt_cvt(band, cc.comp, sd, w, 1, want_mean_ds=False)
    tile = autotune.stats_tile(tuple(band.shape), len(seeds), wl.n_bands, int(x.shape[0]),
                               lambda: L.lsrvt_aggregate(r1.cell, r1.sites, r1.site_comp, cc.comp_band, cc.n_comp,
                                                         wl.n_bands, x, e, cov=True))
    del r1
    _log(f"flame: relaxation grid {grid}, statistics tile {tile} voxels per thread")
    with autotune.shapes(br_grid=grid, stats_tile=tile):
        ms, timing = timed_steps(step, args.steps, args.warmup, "flame")
    ph = step.phases()
    out = {
        "metric": "Gvoxels/s per Lloyd iteration (whole step incl. isobands, components, final pass, stats)",
        "value": round(n * wl.iters / (ms / 1e3) / 1e9, 4), "unit": "Gvoxels/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "flame 1024x512x512 (combustion-shaped sheet), 10 isovalues of Z, |grad T| uint16 "
                               "weights, 1 site / 4096 weighted voxels, T=30, 18 vars (Z, T, 16 species), "
                               "32-bin hist, 18x18 cov",
                   "voxels": n, "iters": wl.iters, "sites": int(len(seeds)), "components": int(cc.n_comp),
                   "parallelism": "single GPU"},
        "phases_ms": ph,
        "lloyd_gvox_per_iter_s": round(n * wl.iters / (ph["lloyd"] / 1e3) / 1e9, 4) if ph["lloyd"] else None,
        "stats_gvox_s": round(n / (ph["aggregate"] / 1e3) / 1e9, 4) if ph["aggregate"] else None,
        "end_to_end_gvox_s": round(n / (ms / 1e3) / 1e9, 4),
        "stats_dtype": "f32 compensated per cell, f64 merges",
        "tuning": {"vt_schedule": "bricks" if timing[4] == 2 else "levels" if timing[4] == 1 else "both",
                   "br_grid": grid, "stats_tile": tile},
        "roofline": roofline(timing, "flame"),
    }
    if not args.no_extras:
        _log("flame: joint moments of the step's cells, 18 variables")
        out["comoments"] = bench_comoments(L, step, cc, x, wl.n_bands, n, reps=1)
        torch.cuda.empty_cache()
    del x, e
    if not args.no_cpu_baseline:
        _log("flame: timing the oracle on a bounded sample")
        z = 16
        out["cpu_baseline"] = cpu_baseline(
            np.ascontiguousarray(wl.field[:z]), wl.iso, np.ascontiguousarray(wl.weights[:z]),
            np.ascontiguousarray(wl.variables[:, :z]), wl.edges, wl.rho, wl.seed, wl.iters,
            f"the first {z} z-planes of the same 1024x512x512 fields (1024x512x{z}, {n * z // 512} voxels, its own "
            f"components and sites)")
    return out


def bench_fourier(args, extras=True):
    """The 256^3 Fourier workload's whole step; with `extras`, the joint
    moments, on-device seeding and the line-of-sight Lloyd loop beside it."""
    import numpy as np
    import torch
    import paper_2208_06970_amd as L
    import synth
    _log("fourier: generating the 256^3 workload")
    wl = synth.fourier_workload(shape=(args.size,) * 3)
    n = wl.field.size
    f = torch.from_numpy(wl.field).cuda()
    w = torch.from_numpy(wl.weights.view(np.int16)).cuda()
    x = torch.from_numpy(np.ascontiguousarray(wl.variables)).cuda()
    e = torch.from_numpy(wl.edges).cuda()
    band, _ = L.lsrvt_isobands(f, wl.iso)
    cc = L.lsrvt_components(band, wl.n_bands)
    seeds = synth.workload_sites(wl, cc.comp.cpu().numpy().view(np.uint32), cc.n_comp)
    sd = torch.from_numpy(seeds.view(np.int32)).cuda()
    step = Step(f, wl.iso, wl.n_bands, sd, w, wl.iters, x, e)
    ms, timing = timed_steps(step, args.steps, args.warmup, "fourier")
    ph = step.phases()
    out = {"value": round(n * wl.iters / (ms / 1e3) / 1e9, 4), "unit": "Gvoxels/s per Lloyd iteration",
           "ms_per_step": round(ms, 3), "steps": args.steps,
           "config": {"workload": f"fourier {args.size}^3, 512 modes k^-5/3, 8 isovalues, |grad| uint16 weights, "
                                  f"1 site / 4096 weighted voxels, T={wl.iters}, 8 vars, 32-bin hist, 8x8 cov",
                      "voxels": n, "iters": wl.iters, "sites": int(len(seeds)), "components": int(cc.n_comp)},
           "phases_ms": ph,
           "lloyd_gvox_per_iter_s": round(n * wl.iters / (ph["lloyd"] / 1e3) / 1e9, 4) if ph["lloyd"] else None,
           "stats_gvox_s": round(n / (ph["aggregate"] / 1e3) / 1e9, 4) if ph["aggregate"] else None,
           "roofline": roofline(timing, "fourier256")}
    if extras:
        out["seeding"] = bench_seeding(L, cc, w, n)
        out["comoments"] = bench_comoments(L, step, cc, x, wl.n_bands, n)
        out["los"] = bench_los(L, cc, sd, w, n, wl.iters)
    return out


def _fourier_job_inputs(shape, seed, n_iso, n_vars, n_bins, rho, n_modes=128):
    """Host arrays of one Fourier job (field, isovalues, weights, variables, edges)."""
    import synth
    return synth.fourier_job(shape, seed, n_iso, n_vars, n_bins, n_modes)


def _device_job(shape, seed, n_iso, n_vars, n_bins, rho, iters):
    """A job with inputs on the device; sites drawn from its components (computed once, outside timing)."""
    import numpy as np
    import torch
    import paper_2208_06970_amd as L
    import synth
    f, iso, w, x, e = _fourier_job_inputs(shape, seed, n_iso, n_vars, n_bins, rho)
    fd = torch.from_numpy(f).cuda()
    band, _ = L.lsrvt_isobands(fd, iso)
    cc = L.lsrvt_components(band, n_iso + 1)
    comp = cc.comp.cpu().numpy().view(np.uint32)
    seeds = synth.seed_sites(comp, cc.n_comp, w, rho, 7919 * seed + 1)
    return dict(field=fd, iso=iso, seeds=torch.from_numpy(seeds.view(np.int32)).cuda(),
                weights=torch.from_numpy(w.view(np.int16)).cuda(), iters=iters,
                variables=torch.from_numpy(x).cuda(), edges=torch.from_numpy(e).cuda(), cov=True,
                cap_comp=int(cc.n_comp) + 16, voxels=f.size)


def bench_batch(args):
    """64 uneven volumes: lsrvt_batch_run on several streams vs one job at a time."""
    import numpy as np
    import torch
    import paper_2208_06970_amd as L
    import synth
    specs = synth.batch_specs(args.batch_jobs, 3)
    _log(f"batch: generating {len(specs)} volumes")
    jobs = [_device_job(sh, sd, k, 8, 32, 4096.0, 15) for sh, sd, k in specs]
    vox_iters = sum(j["voxels"] * j["iters"] for j in jobs)

    def make():
        return [L.BatchJob(field=j["field"], iso=j["iso"], seeds=j["seeds"], weights=j["weights"], iters=j["iters"],
                           variables=j["variables"], edges=j["edges"], cov=True, cap_comp=j["cap_comp"])
                for j in jobs]

    def serial():
        ws = L.Workspace()
        for j in jobs:
            band, _ = L.lsrvt_isobands(j["field"], j["iso"])
            cc = L.lsrvt_components(band, len(j["iso"]) + 1, cap_comp=j["cap_comp"], ws=ws)
            r = L.lsrvt_cvt(band, cc.comp, j["seeds"], j["weights"], j["iters"], ws=ws, want_mean_ds=False)
            L.lsrvt_aggregate(r.cell, r.sites, r.site_comp, cc.comp_band, cc.n_comp, len(j["iso"]) + 1,
                              j["variables"], j["edges"], cov=True, ws=ws)
        torch.cuda.synchronize()

    res = {}
    ws = L.Workspace()
    reps = max(1, min(args.steps, 3))
    from paper_2208_06970_amd import autotune
    streams = autotune.batch_streams(make, key=f"fourier-batch-{len(jobs)}", ws=ws)
    _log(f"batch: autotuned streams = {streams}")
    for name, fn in (("serial", serial), ("batched", lambda: L.lsrvt_batch_run(make(), n_streams=streams, ws=ws))):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        res[name] = float(np.median(ts))
        _log(f"batch {name}: {res[name] * 1e3:.1f} ms")
    return {"metric": "Gvoxels/s per Lloyd iteration, 64-volume batch (whole path per job)",
            "unit": "Gvoxels/s", "value": round(vox_iters / res["batched"] / 1e9, 4),
            "serial_value": round(vox_iters / res["serial"] / 1e9, 4),
            "ms_batched": round(res["batched"] * 1e3, 3), "ms_serial": round(res["serial"] * 1e3, 3),
            "speedup": round(res["serial"] / res["batched"], 3), "streams": streams, "reps": reps,
            "form": "labels and statistics per job on autotuned streams; Lloyd loops of all jobs in lockstep, "
                    "one launch per phase over all jobs",
            "config": {"workload": "64 Fourier volumes, edges 32..192 (cubes and 2:1:1), 3..10 isovalues, "
                                   "T=15, 8 vars, 32-bin hist, 8x8 cov", "voxels": int(sum(j["voxels"] for j in jobs))}}


def serving_jobs(n, seed=5000, pool=6, max_edge=512):
    """Jobs of the serving configuration: per request, edges uniform in
    64..max_edge per axis, 3..12 isovalues, 10..30 updates, 4..16 variables.
    The fields come from a pool of `pool` generated Fourier volumes (one per
    drawn shape, reused by later requests with their own isovalue count,
    update count and variable count) so that generating inputs stays within
    the benchmark's time; each request's variables are smooth functions of
    its field computed on the device."""
    import numpy as np
    import torch
    import paper_2208_06970_amd as L
    import paper_2208_06970_amd.serve as srv
    import synth
    rng = np.random.default_rng(seed)
    vols = []
    for p in range(pool):
        shape = tuple(int(v) for v in rng.integers(64, max_edge + 1, size=3))
        f = synth.fourier_field(shape, seed + p, n_modes=64)
        w = synth.gradient_weight(f)
        vols.append((f, torch.from_numpy(f).cuda(), torch.from_numpy(w.view(np.int16)).cuda(), w))
    jobs = []
    for i in range(n):
        f, fd, wd, w = vols[int(rng.integers(0, pool))]
        K, T, m = int(rng.integers(3, 13)), int(rng.integers(10, 31)), int(rng.integers(4, 17))
        iso = synth.quantile_isovalues(f, [(k + 1) / (K + 1) for k in range(K)])
        band, _ = L.lsrvt_isobands(fd, iso)
        cc = L.lsrvt_components(band, K + 1)
        seeds = synth.seed_sites(cc.comp.cpu().numpy().view(np.uint32), cc.n_comp, w, 4096.0, 7919 * (seed + i) + 1)
        x = torch.stack([torch.sin(fd * (2.0 + j) + 0.5 * j) * (1.0 + j) for j in range(m)]).contiguous()
        lo = x.reshape(m, -1).min(dim=1).values.cpu().numpy()
        hi = x.reshape(m, -1).max(dim=1).values.cpu().numpy()
        edges = np.stack([np.linspace(float(a), float(b), 33) for a, b in zip(lo, hi)]).astype(np.float32)
        jobs.append(srv.Job(field=fd, iso=iso, seeds=torch.from_numpy(seeds.view(np.int32)).cuda(), weights=wd,
                            iters=T, variables=x, edges=torch.from_numpy(edges).cuda(), cov=True,
                            cap_comp=int(cc.n_comp) + 16))
    return jobs


def bench_serve(args, rates=None, n_jobs=None):
    """Poisson arrivals through the serving loop against serial plain launches."""
    import paper_2208_06970_amd.serve as srv
    rates = rates or args.rates
    n_jobs = n_jobs or args.serve_jobs
    _log(f"serve: generating {n_jobs} jobs")
    jobs = serving_jobs(n_jobs, pool=args.serve_pool)
    budget = int(args.budget_gib * 2**30)
    from paper_2208_06970_amd import autotune
    import paper_2208_06970_amd as L
    for j in jobs:  # the Voronoi schedule of every job class, tuned before timing
        band, _ = L.lsrvt_isobands(j.field, j.iso)
        autotune.vt_engine(band, j.seeds, len(j.iso) + 1)
    srv.serve(jobs[:2], [0.0, 0.0], slots=2, budget_bytes=budget)  # warm-up
    vox = [j.voxels for j in jobs]
    out = {"metric": "p50/p99 request latency and throughput, Poisson job stream", "unit": "ms / Gvoxels/s",
           "config": {"workload": f"{len(jobs)} jobs per rate, edges 64..512 per axis (fields from a pool of "
                                  f"{args.serve_pool} volumes), 3..12 isovalues, T=10..30, 4..16 vars, 32-bin hist, cov",
                      "mean_voxels": int(sum(vox) / len(vox)), "budget_gib": args.budget_gib, "slots": args.slots},
           "rates": {}}
    for rate in rates:
        arr = srv.poisson_arrivals(len(jobs), rate, 5)
        a = srv.serve(jobs, arr, slots=args.slots, budget_bytes=budget).summary()
        b = srv.serial(jobs, arr).summary()
        out["rates"][str(rate)] = {"served": a, "serial": {k: b[k] for k in ("makespan_s", "jobs_per_s",
                                                                               "gvox_iter_per_s", "p50_ms", "p99_ms",
                                                                               "mean_ms")}}
        _log(f"serve rate {rate}: p50/p99 {a['p50_ms']} / {a['p99_ms']} ms, {a['gvox_iter_per_s']} Gvox/s "
             f"(serial {b['p50_ms']} / {b['p99_ms']} ms, {b['gvox_iter_per_s']} Gvox/s)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="main line without the c2/batch/serve keys")
    ap.add_argument("--size", type=int, default=256, help="edge of the cubic Fourier volume")
    ap.add_argument("--fourier", action="store_true", help="256^3 Fourier workload (own JSON line)")
    ap.add_argument("--batch", action="store_true", help="64-volume batch vs serial (own JSON line)")
    ap.add_argument("--batch-jobs", type=int, default=64)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--serve", action="store_true", help="Poisson serving loop (own JSON line)")
    ap.add_argument("--serve-jobs", type=int, default=40)
    ap.add_argument("--serve-pool", type=int, default=6)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--rates", type=float, nargs="*", default=[5.0, 10.0, 20.0, 50.0, 100.0, 200.0])
    ap.add_argument("--budget-gib", type=float, default=96.0)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); a multi-GPU layout is "
              "not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.copy_mib:
        src = torch.ones(args.copy_mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "launches": 3}), flush=True)
        return
    if args.batch:
        out = bench_batch(args)
        out.update(n_gpus=1, steps=args.steps, higher_is_better=True, dtype="u32", data="synthetic")
        print(json.dumps(out), flush=True)
        return
    if args.serve:
        out = bench_serve(args)
        out.update(n_gpus=1, dtype="u32", data="synthetic")
        print(json.dumps(out), flush=True)
        return
    if args.fourier:
        f = bench_fourier(args, extras=not args.no_extras)
        out = {"metric": "Gvoxels/s per Lloyd iteration (whole step incl. isobands, components, final pass, stats)",
               "n_gpus": 1, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
               "vs_baseline": None, "dtype": "u32", "data": "synthetic"}
        out.update(f)
        print(json.dumps(out), flush=True)
        return
    out = bench_flame(args)
    torch.cuda.empty_cache()
    if not args.no_extras:
        fargs = argparse.Namespace(**vars(args))
        fargs.steps, fargs.warmup = min(args.steps, 3), 1
        out["fourier256"] = bench_fourier(fargs, extras=False)
        torch.cuda.empty_cache()
        out["batch"] = bench_batch(fargs)
        torch.cuda.empty_cache()
        out["serve"] = bench_serve(fargs, rates=[10.0, 50.0], n_jobs=24)
    print(json.dumps(out), flush=True)


def bench_comoments(L, step, cc, x, n_bands, n, reps: int = 3):
    """Joint moments up to fourth order (lsrvt_comoments) of the cells of one
    step, all variables, timed on their own."""
    import torch
    r, _ = step(False)
    ws = L.Workspace(x.device)
    L.lsrvt_comoments(r.cell, r.sites, r.site_comp, cc.comp_band, cc.n_comp, n_bands, x, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        L.lsrvt_comoments(r.cell, r.sites, r.site_comp, cc.comp_band, cc.n_comp, n_bands, x, ws=ws)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    m = int(x.shape[0])
    units = m + m * (m + 1) // 2 + m * (m + 1) * (m + 2) // 6 + m * (m + 1) * (m + 2) * (m + 3) // 24
    return {"ms": round(ms, 4), "gvox_s": round(n / (ms / 1e3) / 1e9, 4), "vars": m, "sums_per_voxel": units,
            "dtype": "f64", "includes": "structured layout of the cells, merges, host synchronisations"}


def bench_los(L, cc, sd, w, n, iters):
    """The Lloyd loop with the Euclidean line-of-sight tessellation
    (lsrvt_los_cvt: T updates, T + 1 passes) on the step's components, sites
    and weights, one call timed on its own after a single-pass warm-up."""
    import torch
    ws = L.Workspace(w.device)
    r = L.lsrvt_los_cvt(cc.comp, sd, w, 0, ws=ws)
    torch.cuda.synchronize()
    one_pass_sweeps = r.vt.sweeps[0]
    _log("los: timing the line-of-sight Lloyd loop")
    t0 = time.perf_counter()
    r = L.lsrvt_los_cvt(cc.comp, sd, w, iters, ws=ws)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    # roofline of the whole loop against the bytes a pass must move at the
    # least: component ids in (4 B), float64 length, source and cell out
    # (8 + 4 + 4 B) per voxel and pass; the updates ride along in the time
    alg = LOS_BYTES_PER_VOXEL * n * (iters + 1)
    achieved = alg / (ms / 1e3) / 1e9
    return {"ms": round(ms, 3), "iters": iters, "ms_per_pass": round(ms / (iters + 1), 3),
            "gvox_per_iter_s": round(n * iters / (ms / 1e3) / 1e9, 4), "sweeps": int(r.vt.sweeps[0]),
            "sweeps_first_pass": int(one_pass_sweeps), "dtype": "f64 lengths, exact integer update",
            "includes": "host synchronisation every 8 sweeps",
            "roofline": {"bound": "hbm", "kernel": "line-of-sight pass (k_los_mark, k_los_eval, k_los_apply) and update",
                         "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                         "alg_bytes_per_voxel_pass": LOS_BYTES_PER_VOXEL, "passes": iters + 1}}


def bench_seeding(L, cc, w, n, reps: int = 5):
    """On-device stratified initial sites (lsrvt_seed) on the same volume,
    timed on their own (the step above takes its sites as an input)."""
    import torch
    ws = L.Workspace(w.device)
    kw = dict(rho=4096, block=16, seed=0x5EED)
    s = L.lsrvt_seed(cc.comp, cc.comp_first, cc.n_comp, w, None, ws=ws, **kw)  # sizes the workspace
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s = L.lsrvt_seed(cc.comp, cc.comp_first, cc.n_comp, w, None, ws=ws, **kw)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    return {"ms": round(ms, 4), "gvox_s": round(n / (ms / 1e3) / 1e9, 4), "sites": int(s.numel()),
            "rho": kw["rho"], "block": kw["block"], "includes": "two host synchronisations per call"}


if __name__ == "__main__":
    main()
