"""Serving loop on the GPU: jobs admitted by HBM footprint into concurrent
slots, at phase boundaries, give exactly the results they give alone; the
device memory in use (torch's allocated bytes) never exceeds the budget;
latency percentiles are reported.  Two scales: small jobs, and jobs of the
serving configuration's sizes (edges 64..512 per axis, 3..12 isovalues,
10..30 updates, 4..16 variables)."""
import numpy as np
import pytest

import paper_2208_06970_amd as L
import paper_2208_06970_amd.serve as srv
import synth
from tests.gpu_util import banner, dev, host

pytestmark = pytest.mark.gpu


def _jobs(n, seed0=40):
    import oracle
    rng = np.random.default_rng(seed0)
    out = []
    for i in range(n):
        shape = tuple(int(v) for v in rng.integers(12, 40, size=3))
        K = int(rng.integers(3, 9))
        f = synth.fourier_field(shape, seed0 + i, n_modes=32)
        iso = synth.quantile_isovalues(f, [(k + 1) / (K + 1) for k in range(K)])
        w = synth.gradient_weight(f)
        m = int(rng.integers(1, 5))
        x = np.stack([synth.fourier_field(shape, 1000 + 10 * i + j, n_modes=32) for j in range(m)])
        edges = synth.histogram_edges(x, 8)
        cc = oracle.components(oracle.bands(f, iso), K + 1)
        seeds = synth.seed_sites(cc.comp, cc.n_comp, w, 64.0, seed0 + 100 + i)
        out.append(srv.Job(field=dev(f), iso=iso, seeds=dev(seeds), weights=dev(w), iters=int(rng.integers(0, 4)),
                           variables=dev(np.ascontiguousarray(x)), edges=dev(edges), cov=bool(i % 2),
                           cap_comp=int(cc.n_comp) + 8))
    return out


def serving_scale_jobs(n, seed=5000):
    """Jobs of the serving configuration's sizes: a Fourier field (64 modes)
    per job from the input generator; its variables are smooth functions of
    the field computed on the device (deterministic, so alone and mixed runs
    see the same inputs); sites one per 4096 weight-scaled voxels."""
    import torch
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n):
        shape = tuple(int(v) for v in rng.integers(64, 513, size=3))
        K = int(rng.integers(3, 13))
        T = int(rng.integers(10, 31))
        m = int(rng.integers(4, 17))
        f = synth.fourier_field(shape, seed + i, n_modes=64)
        iso = synth.quantile_isovalues(f, [(k + 1) / (K + 1) for k in range(K)])
        w = synth.gradient_weight(f)
        fd, wd = dev(f), dev(w)
        band, _ = L.lsrvt_isobands(fd, iso)
        cc = L.lsrvt_components(band, K + 1)
        comp = host(cc.comp, np.uint32)
        seeds = synth.seed_sites(comp, cc.n_comp, w, 4096.0, 7919 * (seed + i) + 1)
        x = torch.stack([torch.sin(fd * (2.0 + j) + 0.5 * j) * (1.0 + j) for j in range(m)]).contiguous()
        lo, hi = x.reshape(m, -1).min(dim=1).values.cpu().numpy(), x.reshape(m, -1).max(dim=1).values.cpu().numpy()
        edges = np.stack([np.linspace(float(a), float(b), 33) for a, b in zip(lo, hi)]).astype(np.float32)
        jobs.append(srv.Job(field=fd, iso=iso, seeds=dev(seeds), weights=wd, iters=T, variables=x, edges=dev(edges),
                            cov=True, cap_comp=int(cc.n_comp) + 16))
    return jobs


def _same(a, b):
    assert np.array_equal(host(a["band"]), host(b["band"]))
    assert np.array_equal(host(a["comp"].comp), host(b["comp"].comp))
    assert a["comp"].n_comp == b["comp"].n_comp
    for k in ("cell", "sites", "site_comp"):
        assert np.array_equal(host(getattr(a["cvt"], k)), host(getattr(b["cvt"], k))), k
    for la, lb in zip(a["stats"], b["stats"]):
        for k in ("n", "mean", "m2", "vmin", "vmax", "hist", "cov"):
            x, y = getattr(la, k), getattr(lb, k)
            assert (x is None) == (y is None)
            if x is not None:
                assert np.array_equal(host(x), host(y)), k


def _alone_then_mix(jobs, budget, slots, rate, device_check=True):
    """Results alone (one slot, back to back) and in the mix must agree bit
    for bit.  Kept results belong to the caller and are not part of the
    budget, so the device-bytes bound is checked on a run that drops them."""
    alone = srv.serve(jobs, [0.0] * len(jobs), slots=1, budget_bytes=budget, keep_results=True)
    ref = [j.result for j in jobs]
    assert alone.peak_bytes <= budget
    arr = srv.poisson_arrivals(len(jobs), rate, 5)
    if device_check:
        free = srv.serve(jobs, arr, slots=slots, budget_bytes=budget)
        assert free.peak_bytes <= budget, (free.peak_bytes, budget)
        assert free.peak_device_bytes <= budget, (free.peak_device_bytes, budget)
    mix = srv.serve(jobs, arr, slots=slots, budget_bytes=budget, keep_results=True)
    assert mix.peak_bytes <= budget, (mix.peak_bytes, budget)
    assert mix.statuses == {"done": len(jobs)}
    for r0, j in zip(ref, jobs):
        _same(r0, j.result)
    s = mix.summary()
    assert s["p50_ms"] is not None and s["p99_ms"] >= s["p50_ms"]
    return s


def test_serving_alone_equals_mix_and_budget():
    jobs = _jobs(8)
    banner("serve: 8 small jobs alone, then Poisson arrivals on 3 slots")
    budget = 4 * max(j.footprint() for j in jobs)
    s = _alone_then_mix(jobs, budget, 3, 200.0)
    banner(f"serve: {s}")


def test_serving_tight_budget_serialises():
    jobs = _jobs(4, seed0=70)
    budget = max(j.footprint() for j in jobs)  # room for one job at a time
    banner("serve: tight budget")
    rep = srv.serve(jobs, [0.0] * len(jobs), slots=4, budget_bytes=budget)
    assert rep.peak_bytes <= budget and rep.peak_device_bytes <= budget
    with pytest.raises(ValueError):
        srv.serve(jobs, [0.0] * len(jobs), slots=2, budget_bytes=budget // 4)


def test_serving_invalid_job_fails_alone():
    jobs = _jobs(3, seed0=90)
    bad = jobs[1]
    import torch
    bad.seeds = torch.full_like(bad.seeds, 2**30)        # a seed outside the volume: the library rejects it
    banner("serve: one invalid job among three")
    rep = srv.serve(jobs, [0.0] * 3, slots=2, budget_bytes=4 * max(j.footprint() for j in jobs), keep_results=True)
    assert rep.statuses == {"done": 2, "failed": 1}
    assert jobs[1].status == "failed" and jobs[0].status == "done" and jobs[2].status == "done"


def test_serving_scale_alone_equals_mix():
    jobs = serving_scale_jobs(4)
    vox = [j.voxels for j in jobs]
    banner(f"serve scale: 4 jobs, voxels {vox}")
    budget = 2 * max(j.footprint() for j in jobs)
    s = _alone_then_mix(jobs, budget, 3, 50.0, device_check=False)
    banner(f"serve scale: {s}")
