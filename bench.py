"""Benchmark of the level-set restricted Voronoi hot path on one MI355X.

One step = the whole hot path over one synthetic volume, with all inputs
already resident in HBM: isobands -> components -> Lloyd loop (T updates and
T + 1 restricted geodesic Voronoi passes) -> statistics of every cell merged to
components and bands.  The initial sites are an input of the Lloyd loop; they
are drawn once before timing from the (deterministic) components.

Default workload: the 256^3 turbulence-like Fourier field (8 isovalues at
quantiles, |grad f| saliency weights as uint16, one site per 4096
weight-scaled voxels, 20 updates, 8 statistics variables with 32-bin
histograms and the full 8x8 covariance).

value = voxels * T / step time, in Gvoxels/s per Lloyd iteration, with the
whole step (isobands, components, final pass and statistics included) in the
denominator.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--flame | --batch | --serve]

The main line also carries, timed on their own outside the step, the
on-device stratified initial sites of the same volume ("seeding"), the
joint moments up to fourth order of the step's cells ("comoments") and the
Lloyd loop with the Euclidean line-of-sight tessellation and the ray-clamped
site update on the same components, sites and T ("los").

Three more modes print their own JSON line instead of the main one:
  --flame   the combustion-shaped 1024 x 512 x 512 volume (10 isovalues of
            the mixture fraction, |grad T| weights, 30 updates, 18 variables
            with 32-bin histograms and the 18 x 18 covariance), whole step;
  --batch   64 independent Fourier volumes (edges 32..192, cubes and 2:1:1
            boxes, 3..10 isovalues, 15 updates) through lsrvt_batch_run on
            several streams, against the same jobs run one at a time;
  --serve   a Poisson stream of jobs (edges 64..192 per axis, 3..12
            isovalues, 10..30 updates, 4..8 variables) through the serving
            loop with HBM-footprint admission, against one slot; reports
            p50/p99 latency and throughput per arrival rate.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_bfs_level_traffic.json")
CVT_SOURCE = os.path.join(ROOT, "paper_2208_06970_amd", "csrc", "cvt.hip")


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _source_hash():
    with open(CVT_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic_per_launch():
    """HBM bytes per launch of the Voronoi level kernel from committed rocprofv3 counters,
    or None when they are missing or the kernel source changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256_16") != _source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(wl, seeds, T_sample=2):
    """The oracle as it stands, single-threaded, on the same volume with
    T_sample updates (a bounded sample of the step)."""
    import oracle
    import numpy as np
    t0 = time.perf_counter()
    band = oracle.bands(wl.field, wl.iso)
    cc = oracle.components(band, wl.n_bands)
    r = oracle.cvt(cc.comp, seeds, wl.weights, T_sample)
    S = len(seeds)
    oracle.stats(r.cell, S, wl.variables, wl.edges, cov=True)
    comp_unit = np.where(r.cell == oracle.NONE_ID, oracle.NONE_ID, r.site_comp[np.minimum(r.cell, S - 1)])
    oracle.stats(comp_unit.astype(np.uint32), cc.n_comp, wl.variables, wl.edges, cov=True)
    band_unit = np.where(r.cell == oracle.NONE_ID, oracle.NONE_ID, band.astype(np.uint32))
    oracle.stats(band_unit.astype(np.uint32), wl.n_bands, wl.variables, wl.edges, cov=True)
    dt = time.perf_counter() - t0
    n = wl.field.size
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": n * T_sample / dt / 1e9, "unit": "Gvoxels/s per Lloyd iteration", "cores": 1,
            "kind": "oracle", "seconds": round(dt, 3), "host_cpu": model,
            "host_threads": len(os.sched_getaffinity(0)),
            "sample": f"same {wl.field.shape[2]}x{wl.field.shape[1]}x{wl.field.shape[0]} volume, full pipeline "
                      f"(isobands, components, Lloyd loop, three-level statistics) with {T_sample} updates "
                      f"instead of {wl.iters}; single-threaded C"}


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
    for name, fn in (("serial", serial), ("batched", lambda: L.lsrvt_batch_run(make(), n_streams=args.streams, ws=ws))):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        res[name] = float(np.median(ts))
        _log(f"batch {name}: {res[name] * 1e3:.1f} ms")
    print(json.dumps({"metric": "Gvoxels/s per Lloyd iteration, 64-volume batch (whole path per job)",
                      "unit": "Gvoxels/s", "higher_is_better": True, "n_gpus": 1, "steps": args.steps,
                      "value": round(vox_iters / res["batched"] / 1e9, 4),
                      "serial_value": round(vox_iters / res["serial"] / 1e9, 4),
                      "ms_batched": round(res["batched"] * 1e3, 3), "ms_serial": round(res["serial"] * 1e3, 3),
                      "speedup": round(res["serial"] / res["batched"], 3), "streams": args.streams,
                      "config": {"workload": "64 Fourier volumes, edges 32..192 (cubes and 2:1:1), 3..10 isovalues, "
                                             "T=15, 8 vars, 32-bin hist, 8x8 cov", "voxels": int(sum(j["voxels"] for j in jobs))},
                      "dtype": "u32", "data": "synthetic"}), flush=True)


def bench_serve(args):
    """Poisson arrivals through the serving loop, several slots vs one slot."""
    import numpy as np
    import paper_2208_06970_amd.serve as srv
    rng = np.random.default_rng(5)
    specs = []
    for j in range(args.serve_jobs):
        shape = tuple(int(v) for v in rng.integers(64, 193, size=3))
        specs.append((shape, 5000 + j, int(rng.integers(3, 13)), int(rng.integers(4, 9)), int(rng.integers(10, 31))))
    _log(f"serve: generating {len(specs)} jobs")
    made = [_device_job(sh, sd, k, m, 32, 4096.0, t) for sh, sd, k, m, t in specs]
    jobs = [srv.Job(field=d["field"], iso=d["iso"], seeds=d["seeds"], weights=d["weights"], iters=d["iters"],
                    variables=d["variables"], edges=d["edges"], cov=True, cap_comp=d["cap_comp"]) for d in made]
    budget = int(args.budget_gib * 2**30)
    srv.serve(jobs[:2], [0.0, 0.0], slots=2, budget_bytes=budget)  # warm-up
    out = {"metric": "p50/p99 request latency and throughput, Poisson job stream", "unit": "ms / Gvoxels/s",
           "n_gpus": 1, "data": "synthetic", "dtype": "u32",
           "config": {"workload": f"{len(jobs)} jobs, edges 64..192 per axis, 3..12 isovalues, T=10..30, 4..8 vars, "
                                  f"32-bin hist, cov", "budget_gib": args.budget_gib, "slots": args.slots},
           "rates": {}}
    for rate in args.rates:
        arr = srv.poisson_arrivals(len(jobs), rate, 5)
        a = srv.serve(jobs, arr, slots=args.slots, budget_bytes=budget).summary()
        b = srv.serve(jobs, arr, slots=1, budget_bytes=budget).summary()
        out["rates"][str(rate)] = {"served": a, "one_slot": b}
        _log(f"serve rate {rate}: {a['p50_ms']} / {a['p99_ms']} ms (one slot {b['p50_ms']} / {b['p99_ms']})")
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--size", type=int, default=256, help="edge of the cubic Fourier volume")
    ap.add_argument("--batch", action="store_true", help="64-volume batch vs serial (own JSON line)")
    ap.add_argument("--batch-jobs", type=int, default=64)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--serve", action="store_true", help="Poisson serving loop (own JSON line)")
    ap.add_argument("--flame", action="store_true", help="1024x512x512 combustion-shaped volume (own JSON line)")
    ap.add_argument("--serve-jobs", type=int, default=24)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--rates", type=float, nargs="*", default=[5.0, 20.0, 50.0])
    ap.add_argument("--budget-gib", type=float, default=96.0)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); a multi-GPU layout is "
              "not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2208_06970_amd as L
    import synth

    torch.cuda.set_device(0)
    if args.batch:
        bench_batch(args)
        return
    if args.serve:
        bench_serve(args)
        return
    if args.flame:
        bench_flame(args)
        return
    if args.copy_mib:
        src = torch.ones(args.copy_mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "launches": 3}), flush=True)
        return
    _log("generating workload")
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
    _log(f"volume {wl.field.shape} comps={cc.n_comp} sites={len(seeds)}")

    ev = {k: torch.cuda.Event(enable_timing=True) for k in ("t0", "t1", "t2", "t3", "t4")}
    phase_ms = {"isobands": 0.0, "components": 0.0, "lloyd": 0.0, "aggregate": 0.0}

    def step(record):
        if record:
            ev["t0"].record()
        b, _ = L.lsrvt_isobands(f, wl.iso)
        if record:
            ev["t1"].record()
        c = L.lsrvt_components(b, wl.n_bands)
        if record:
            ev["t2"].record()
        r = L.lsrvt_cvt(b, c.comp, sd, w, wl.iters, want_mean_ds=False)
        if record:
            ev["t3"].record()
        L.lsrvt_aggregate(r.cell, r.sites, r.site_comp, c.comp_band, c.n_comp, wl.n_bands, x, e, cov=True)
        if record:
            ev["t4"].record()
            torch.cuda.synchronize()
            phase_ms["isobands"] += ev["t0"].elapsed_time(ev["t1"])
            phase_ms["components"] += ev["t1"].elapsed_time(ev["t2"])
            phase_ms["lloyd"] += ev["t2"].elapsed_time(ev["t3"])
            phase_ms["aggregate"] += ev["t3"].elapsed_time(ev["t4"])
        return r

    for i in range(args.warmup):
        step(False)
        _log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    L.lsrvt_timing_read()                      # discard anything recorded so far
    L.lsrvt_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
        _log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    L.lsrvt_timing_enable(False)
    vt_ms, vt_launches, vt_passes, vox_per_pass = L.lsrvt_timing_read()

    ms_per_step = dt * 1e3 / args.steps
    value = n * wl.iters / (ms_per_step / 1e3) / 1e9
    phases = {k: round(v / args.steps, 4) for k, v in phase_ms.items()}
    # roofline of the dominant kernel: the Voronoi level kernel, HBM-bound
    alg_bytes_per_launch = VT_BYTES_PER_VOXEL * vox_per_pass * vt_passes / max(vt_launches, 1)
    avg_launch_s = vt_ms / 1e3 / max(vt_launches, 1)
    achieved = alg_bytes_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    traffic = _traffic_per_launch()
    out = {
        "metric": "Gvoxels/s per Lloyd iteration (whole step incl. isobands, components, final pass, stats)",
        "value": round(value, 4),
        "unit": "Gvoxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"fourier {args.size}^3, 512 modes k^-5/3, 8 isovalues, |grad| uint16 weights, "
                               f"1 site / 4096 weighted voxels, T={wl.iters}, 8 vars, 32-bin hist, 8x8 cov",
                   "voxels": n, "iters": wl.iters, "sites": int(len(seeds)), "components": int(cc.n_comp),
                   "parallelism": "single GPU"},
        "phases_ms": phases,
        "lloyd_gvox_per_iter_s": round(n * wl.iters / (phases["lloyd"] / 1e3) / 1e9, 4) if phases["lloyd"] else None,
        "stats_gvox_s": round(n / (phases["aggregate"] / 1e3) / 1e9, 4) if phases["aggregate"] else None,
        "end_to_end_gvox_s": round(n / (ms_per_step / 1e3) / 1e9, 4),
        "stats_dtype": "f32 compensated per cell, f64 merges",
        "roofline": {"bound": "hbm", "kernel": "k_bfs_level", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": traffic,
                     "avg_launch_us": round(avg_launch_s * 1e6, 3), "launches": vt_launches, "passes": vt_passes,
                     "alg_bytes_per_launch": round(alg_bytes_per_launch, 1)},
    }
    out["seeding"] = bench_seeding(L, cc, w, n)
    out["comoments"] = bench_comoments(L, step, cc, x, wl.n_bands, n)
    out["los"] = bench_los(L, cc, sd, w, n, wl.iters)
    if not args.no_cpu_baseline:
        _log("timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(wl, seeds)
    print(json.dumps(out), flush=True)


def bench_comoments(L, step, cc, x, n_bands, n, reps: int = 3):
    """Joint moments up to fourth order (lsrvt_comoments) of the cells of one
    step, all 8 variables, timed on their own."""
    import torch
    r = step(False)
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


def bench_flame(args):
    """The whole step on the combustion-shaped 1024 x 512 x 512 volume."""
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
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    ph = np.zeros(4)

    def step(record):
        if record:
            ev[0].record()
        b, _ = L.lsrvt_isobands(f, wl.iso)
        if record:
            ev[1].record()
        c = L.lsrvt_components(b, wl.n_bands)
        if record:
            ev[2].record()
        r = L.lsrvt_cvt(b, c.comp, sd, w, wl.iters, want_mean_ds=False)
        if record:
            ev[3].record()
        L.lsrvt_aggregate(r.cell, r.sites, r.site_comp, c.comp_band, c.n_comp, wl.n_bands, x, e, cov=True)
        if record:
            ev[4].record()
            torch.cuda.synchronize()
            for k in range(4):
                ph[k] += ev[k].elapsed_time(ev[k + 1])

    steps = max(1, min(args.steps, 3))
    step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(True)
        _log(f"flame: step {i + 1}/{steps} done")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    ph /= steps
    print(json.dumps({"metric": "Gvoxels/s per Lloyd iteration (whole step incl. isobands, components, final pass, stats)",
                      "value": round(n * wl.iters / (ms / 1e3) / 1e9, 4), "unit": "Gvoxels/s", "n_gpus": 1,
                      "steps": steps, "warmup": 1, "ms_per_step": round(ms, 3), "higher_is_better": True,
                      "dtype": "u32", "data": "synthetic",
                      "config": {"workload": "flame 1024x512x512, 10 isovalues of Z, |grad T| uint16 weights, T=30, "
                                             "18 vars, 32-bin hist, 18x18 cov", "voxels": n, "iters": wl.iters,
                                 "sites": int(len(seeds)), "components": int(cc.n_comp)},
                      "phases_ms": {k: round(float(v), 3) for k, v in zip(("isobands", "components", "lloyd",
                                                                             "aggregate"), ph)},
                      "lloyd_gvox_per_iter_s": round(n * wl.iters / (ph[2] / 1e3) / 1e9, 4),
                      "stats_gvox_s": round(n / (ph[3] / 1e3) / 1e9, 4)}), flush=True)


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
    return {"ms": round(ms, 3), "iters": iters, "ms_per_pass": round(ms / (iters + 1), 3),
            "gvox_per_iter_s": round(n * iters / (ms / 1e3) / 1e9, 4), "sweeps": int(r.vt.sweeps[0]),
            "sweeps_first_pass": int(one_pass_sweeps), "dtype": "f64 lengths, exact integer update",
            "includes": "host synchronisation every 8 sweeps"}


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
