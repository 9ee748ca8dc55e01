"""Serving loop: jobs admitted by HBM footprint into concurrent slots give
exactly the results they give alone, the resident footprint never exceeds the
budget, and latency percentiles are reported."""
import numpy as np
import pytest

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


def _same(a, b):
    for k in ("band",):
        assert np.array_equal(host(a[k]), host(b[k]))
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


def test_serving_alone_equals_mix_and_budget():
    jobs = _jobs(8)
    banner("serve: 8 jobs alone (one slot, back to back)")
    budget = 4 * max(j.footprint() for j in jobs)
    alone = srv.serve(jobs, [0.0] * len(jobs), slots=1, budget_bytes=budget, keep_results=True)
    ref = [j.result for j in jobs]
    assert alone.peak_bytes <= budget
    banner("serve: same jobs, Poisson arrivals, 3 slots")
    mix = srv.serve(jobs, srv.poisson_arrivals(len(jobs), 200.0, 5), slots=3, budget_bytes=budget,
                    keep_results=True)
    assert mix.peak_bytes <= budget
    for r0, j in zip(ref, jobs):
        _same(r0, j.result)
    s = mix.summary()
    assert s["p50_ms"] is not None and s["p99_ms"] >= s["p50_ms"]
    banner(f"serve: {s}")


def test_serving_tight_budget_serialises():
    jobs = _jobs(4, seed0=70)
    budget = max(j.footprint() for j in jobs)  # room for one job at a time
    banner("serve: tight budget")
    rep = srv.serve(jobs, [0.0] * len(jobs), slots=4, budget_bytes=budget)
    assert rep.peak_bytes <= budget
    with pytest.raises(ValueError):
        srv.serve(jobs, [0.0] * len(jobs), slots=2, budget_bytes=budget // 4)
