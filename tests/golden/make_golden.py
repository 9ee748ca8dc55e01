"""Write the oracle's expected results for the full-size workloads.

Calls only the CPU oracle (``oracle``) and the seeded input generators
(``synth``); nothing here runs or reads the GPU library.  Each workload is run
through Algorithm 1 with its configured number of updates (the oracle's
pruned per-site breadth-first search, exact integer centroid and snap), and
its statistics are computed directly per unit in float64 (Sec. 3.3).  The
results are stored as SHA-256 digests of the label arrays (little-endian
bytes in linear order), digests per z-slab (to localise a mismatch) and, for
the statistics, small float64 arrays.

    python tests/golden/make_golden.py fourier   # 256^3 Fourier field, T = 20
    python tests/golden/make_golden.py batch     # the 64-volume batch, T = 15
    python tests/golden/make_golden.py flame     # 1024 x 512 x 512 flame sheet, T = 30

Outputs (next to this file): ``<name>.json`` with the digests and the mean
site displacement of every update, ``<name>_stats.npz`` with component and
band statistics.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

NONE = oracle.NONE_ID
STAT_KEYS = ("n", "mean", "m2", "vmin", "vmax", "hist", "cov")


def sha(a) -> str:
    """SHA-256 of an array's little-endian bytes in C order."""
    a = np.ascontiguousarray(a)
    return hashlib.sha256(a.astype(a.dtype.newbyteorder("<"), copy=False).tobytes()).hexdigest()


def slab_digests(cell: np.ndarray, n_slabs: int):
    """Digests of consecutive z-slabs of a [nz, ny, nx] label array."""
    nz = cell.shape[0]
    bounds = np.linspace(0, nz, min(n_slabs, nz) + 1).astype(int)
    return [[int(a), int(b), sha(cell[a:b])] for a, b in zip(bounds[:-1], bounds[1:])]


def unit_labels(cell, site_comp, comp_band=None, band=None):
    """Component (or band) of every labelled voxel, NONE elsewhere."""
    c = cell.ravel()
    lab = c != NONE
    out = np.full(c.shape, NONE, dtype=np.uint32)
    if band is None:
        out[lab] = site_comp[c[lab]]
    else:
        out[lab] = band.ravel()[lab]
    return out.reshape(cell.shape)


def exact_digests(st) -> dict:
    return {k: sha(getattr(st, k)) for k in ("n", "vmin", "vmax", "hist") if getattr(st, k) is not None}


def stats_arrays(prefix: str, st, rows=None) -> dict:
    out = {}
    for k in STAT_KEYS:
        a = getattr(st, k)
        if a is None:
            continue
        out[f"{prefix}_{k}"] = a if rows is None else a[rows]
    return out


def run_labels(comp, seeds, weights, iters):
    t = time.time()
    r = oracle.cvt(comp, seeds, weights, iters)
    print(f"  oracle Lloyd loop, {iters} updates: {time.time() - t:.1f} s", flush=True)
    return r


def fourier(out_name="fourier256_t20"):
    """The 256^3 Fourier workload (8 isovalues, |grad| weights, one site per
    4096 weight-scaled voxels, 20 updates, 8 variables, 32 bins, covariance)."""
    wl = synth.fourier_workload()
    band = oracle.bands(wl.field, wl.iso)
    cc = oracle.components(band, wl.n_bands)
    seeds = synth.workload_sites(wl, cc.comp, cc.n_comp)
    print(f"fourier 256^3: comps={cc.n_comp} sites={len(seeds)}", flush=True)
    r = run_labels(cc.comp, seeds, wl.weights, wl.iters)
    x = np.ascontiguousarray(wl.variables)
    cu = unit_labels(r.cell, r.site_comp)
    t = time.time()
    gst = oracle.stats(cu, cc.n_comp, x, wl.edges, cov=True)
    bst = oracle.stats(unit_labels(r.cell, r.site_comp, band=band), wl.n_bands, x, wl.edges, cov=True)
    print(f"  oracle statistics: {time.time() - t:.1f} s", flush=True)
    size = gst.n.astype(np.int64)
    top = np.sort(np.argsort(-size, kind="stable")[:256])
    doc = {
        "workload": "fourier 256^3, seed 2, 512 modes, 8 isovalues at quantiles i/9, |grad f| uint16 weights, "
                    "one site per 4096 weight-scaled voxels, 20 updates, 8 variables, 32 bins, covariance",
        "iters": wl.iters, "n_comp": int(cc.n_comp), "n_sites": int(len(seeds)),
        "seeds_sha256": sha(seeds),
        "cell_sha256": sha(r.cell), "sites_sha256": sha(r.sites), "site_comp_sha256": sha(r.site_comp),
        "cell_slabs": slab_digests(r.cell, 64),
        "mean_ds": [float(v) for v in r.mean_ds],
        "comp_exact_sha256": exact_digests(gst), "band_exact_sha256": exact_digests(bst),
    }
    arrays = {"comp_rows": top.astype(np.int64)}
    arrays.update(stats_arrays("comp", gst, top))
    arrays.update(stats_arrays("band", bst))
    write(out_name, doc, arrays)


def flame(out_name="flame_t30"):
    """The combustion-shaped 1024 x 512 x 512 workload (10 isovalues of Z,
    |grad T| weights, 30 updates, 18 variables, 32 bins, covariance)."""
    t = time.time()
    wl = synth.flame_workload()
    print(f"flame: generated in {time.time() - t:.1f} s", flush=True)
    band = oracle.bands(wl.field, wl.iso)
    cc = oracle.components(band, wl.n_bands)
    seeds = synth.flame_sites(cc.comp, cc.n_comp, wl.weights, wl.rho, wl.seed)
    print(f"flame: comps={cc.n_comp} sites={len(seeds)}", flush=True)
    r = run_labels(cc.comp, seeds, wl.weights, wl.iters)
    comp_cell_sha = []
    cflat, kflat = r.cell.ravel(), cc.comp.ravel()
    order = np.argsort(kflat, kind="stable")
    bounds = np.searchsorted(kflat[order], np.arange(cc.n_comp + 1))
    for c in range(cc.n_comp):
        comp_cell_sha.append(sha(cflat[order[bounds[c]:bounds[c + 1]]]))
    del order
    t = time.time()
    x = wl.variables
    gst = oracle.stats(unit_labels(r.cell, r.site_comp), cc.n_comp, x, wl.edges, cov=True)
    bst = oracle.stats(unit_labels(r.cell, r.site_comp, band=band), wl.n_bands, x, wl.edges, cov=True)
    print(f"  oracle statistics: {time.time() - t:.1f} s", flush=True)
    doc = {
        "workload": "flame 1024x512x512 (nx, ny, nz), seed 4, 10 isovalues of Z at 0.05..0.95, |grad T| uint16 "
                    "weights, one site per 4096 weight-scaled voxels (independent draws), 30 updates, 18 variables, "
                    "32 bins, covariance",
        "iters": wl.iters, "n_comp": int(cc.n_comp), "n_sites": int(len(seeds)),
        "seeds_sha256": sha(seeds),
        "cell_sha256": sha(r.cell), "sites_sha256": sha(r.sites), "site_comp_sha256": sha(r.site_comp),
        "cell_slabs": slab_digests(r.cell, 64),
        "comp_cell_sha256": comp_cell_sha,
        "mean_ds": [float(v) for v in r.mean_ds],
        "comp_exact_sha256": exact_digests(gst), "band_exact_sha256": exact_digests(bst),
    }
    arrays = {"comp_rows": np.arange(cc.n_comp, dtype=np.int64)}
    arrays.update(stats_arrays("comp", gst))
    arrays.update(stats_arrays("band", bst))
    write(out_name, doc, arrays)


def batch(out_name="batch64_t15"):
    """The 64-volume batch (long edges 32..192, cubes and 2:1:1 boxes, 3..10
    isovalues, 15 updates, one site per 4096 weight-scaled voxels): labels of
    every job."""
    jobs = []
    for j, (shape, seed, k) in enumerate(synth.batch_specs(64, 3)):
        f, iso, w, x, e = synth.fourier_job(shape, seed, k)
        band = oracle.bands(f, iso)
        cc = oracle.components(band, k + 1)
        seeds = synth.seed_sites(cc.comp, cc.n_comp, w, 4096.0, 7919 * seed + 1)
        print(f"job {j} {shape}: comps={cc.n_comp} sites={len(seeds)}", flush=True)
        r = run_labels(cc.comp, seeds, w, 15)
        jobs.append({"shape": list(shape), "seed": seed, "n_iso": k, "n_comp": int(cc.n_comp),
                     "n_sites": int(len(seeds)), "seeds_sha256": sha(seeds), "cell_sha256": sha(r.cell),
                     "sites_sha256": sha(r.sites), "site_comp_sha256": sha(r.site_comp),
                     "cell_slabs": slab_digests(r.cell, 8), "mean_ds": [float(v) for v in r.mean_ds]})
    write(out_name, {"workload": "64 Fourier volumes (128 modes), batch_specs(64, seed 3), 15 updates",
                     "iters": 15, "jobs": jobs}, None)


def write(name, doc, arrays):
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(doc, fh, indent=1)
        fh.write("\n")
    if arrays:
        np.savez_compressed(os.path.join(HERE, name + "_stats.npz"), **arrays)
    print(f"wrote {name}", flush=True)


if __name__ == "__main__":
    oracle.build()
    for which in sys.argv[1:] or ["fourier", "batch", "flame"]:
        {"fourier": fourier, "batch": batch, "flame": flame}[which]()
