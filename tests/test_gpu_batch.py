"""Many jobs in one call (lsrvt_batch_run): every job's outputs must be
bit-identical to running its four calls alone, whatever else shares the
GPU, and its labels must match the oracle."""
import numpy as np
import pytest

import oracle
import paper_2208_06970_amd as L
import synth
from tests.gpu_util import banner, dev, host

pytestmark = pytest.mark.gpu


def _job(shape, seed, n_iso, iters, m, bins, cov, rho):
    f = synth.fourier_field(shape, seed, n_modes=48)
    iso = synth.quantile_isovalues(f, [(i + 1) / (n_iso + 1) for i in range(n_iso)])
    w = synth.gradient_weight(f)
    x = np.stack([synth.fourier_field(shape, 100 * seed + j, n_modes=48) for j in range(m)])
    edges = None
    if bins:
        edges = np.stack([np.linspace(x[j].min(), x[j].max(), bins + 1) for j in range(m)]).astype(np.float32)
    band = oracle.bands(f, iso)
    cc = oracle.components(band, n_iso + 1)
    seeds = synth.seed_sites(cc.comp, cc.n_comp, w, rho, seed + 7)
    return dict(f=f, iso=iso, w=w, x=x, edges=edges, seeds=seeds, iters=iters, cov=cov, cc=cc, band=band)


def _alone(d):
    f, w, x = dev(d["f"]), dev(d["w"]), dev(np.ascontiguousarray(d["x"]))
    e = None if d["edges"] is None else dev(d["edges"])
    band, _ = L.lsrvt_isobands(f, d["iso"])
    cc = L.lsrvt_components(band, len(d["iso"]) + 1)
    r = L.lsrvt_cvt(band, cc.comp, dev(d["seeds"]), w, d["iters"], want_mean_ds=False)
    st = L.lsrvt_aggregate(r.cell, r.sites, r.site_comp, cc.comp_band, cc.n_comp, len(d["iso"]) + 1, x, e, cov=d["cov"])
    return band, cc, r, st


SPECS = [((24, 40, 32), 1, 3, 3, 2, 16, False, 64.0),
         ((48, 16, 40), 2, 5, 2, 4, 8, True, 96.0),
         ((32, 32, 32), 3, 8, 4, 3, 0, True, 48.0),
         ((17, 50, 29), 4, 2, 1, 1, 12, False, 128.0),
         ((40, 40, 8), 5, 6, 0, 2, 16, True, 80.0),
         ((64, 20, 20), 6, 4, 5, 5, 4, False, 200.0)]


def test_batch_matches_alone_and_oracle():
    data = [_job(*sp) for sp in SPECS]
    alone = []
    for i, d in enumerate(data):
        banner(f"batch: job {i} alone {d['f'].shape}")
        alone.append(_alone(d))
    jobs = [L.BatchJob(field=dev(d["f"]), iso=d["iso"], seeds=dev(d["seeds"]), weights=dev(d["w"]), iters=d["iters"],
                       variables=dev(np.ascontiguousarray(d["x"])),
                       edges=None if d["edges"] is None else dev(d["edges"]), cov=d["cov"],
                       cap_comp=int(d["cc"].n_comp) + 5)
            for d in data]
    banner(f"batch: {len(jobs)} jobs on 3 streams")
    L.lsrvt_batch_run(jobs, n_streams=3)
    for i, (d, j, (band, cc, r, st)) in enumerate(zip(data, jobs, alone)):
        assert j.status == 0 and j.n_comp == cc.n_comp, i
        np.testing.assert_array_equal(host(j.band), host(band))
        np.testing.assert_array_equal(host(j.comp), host(cc.comp))
        np.testing.assert_array_equal(host(j.comp_band)[:j.n_comp], host(cc.comp_band))
        np.testing.assert_array_equal(host(j.comp_size)[:j.n_comp], host(cc.comp_size))
        np.testing.assert_array_equal(host(j.cell), host(r.cell))
        S = len(d["seeds"])
        np.testing.assert_array_equal(host(j.sites)[:S], host(r.sites))
        np.testing.assert_array_equal(host(j.site_comp)[:S], host(r.site_comp))
        for lvl, (a, b) in enumerate(zip(j.stats, st)):
            units = j.n_comp if lvl == 1 else None
            for k in ("n", "mean", "m2", "vmin", "vmax", "hist", "cov"):
                ga, gb = getattr(a, k), getattr(b, k)
                if ga is None:
                    assert gb is None
                    continue
                ga = host(ga)[:units] if units is not None else host(ga)
                assert np.array_equal(ga, host(gb)), (i, lvl, k)
        # labels against the oracle
        np.testing.assert_array_equal(host(j.band), d["band"])
        np.testing.assert_array_equal(host(j.comp, np.uint32), d["cc"].comp)
        want = oracle.cvt(d["cc"].comp, d["seeds"], d["w"], d["iters"])
        np.testing.assert_array_equal(host(j.cell, np.uint32), want.cell)
        np.testing.assert_array_equal(host(j.sites, np.uint32)[:S], want.sites)


@pytest.mark.parametrize("bits", [64, 30])
def test_batch_key_widths(bits):
    """The lockstep Lloyd loops with wide keys, and with narrow keys whose
    distance field every job outgrows (the batch is then run again with wide
    keys): cells and sites as the oracle's."""
    data = [_job(*sp) for sp in SPECS[:4]]
    jobs = [L.BatchJob(field=dev(d["f"]), iso=d["iso"], seeds=dev(d["seeds"]), weights=dev(d["w"]), iters=d["iters"],
                       variables=dev(np.ascontiguousarray(d["x"])),
                       edges=None if d["edges"] is None else dev(d["edges"]), cov=d["cov"],
                       cap_comp=int(d["cc"].n_comp) + 5)
            for d in data]
    banner(f"batch: {len(jobs)} jobs, key bits {bits}")
    prev = L.lsrvt_set_tuning(L.TUNE_KEY_BITS, bits)
    try:
        L.lsrvt_batch_run(jobs, n_streams=2)
    finally:
        L.lsrvt_set_tuning(L.TUNE_KEY_BITS, prev)
    for i, (d, j) in enumerate(zip(data, jobs)):
        assert j.status == 0, i
        want = oracle.cvt(d["cc"].comp, d["seeds"], d["w"], d["iters"])
        np.testing.assert_array_equal(host(j.cell, np.uint32), want.cell)
        np.testing.assert_array_equal(host(j.sites, np.uint32)[:len(d["seeds"])], want.sites)


def test_batch_capacity_and_validation():
    d = _job((20, 20, 20), 9, 4, 1, 1, 0, False, 64.0)
    banner("batch: capacity")
    small = L.BatchJob(field=dev(d["f"]), iso=d["iso"], seeds=dev(d["seeds"]), weights=None, iters=1,
                       variables=dev(np.ascontiguousarray(d["x"])), cap_comp=1)
    ok = L.BatchJob(field=dev(d["f"]), iso=d["iso"], seeds=dev(d["seeds"]), weights=None, iters=1,
                    variables=dev(np.ascontiguousarray(d["x"])), cap_comp=int(d["cc"].n_comp))
    if d["cc"].n_comp > 1:
        with pytest.raises(L.LsrvtError):
            L.lsrvt_batch_run([small, ok], n_streams=2)
        assert small.status == L.ECAPACITY and small.n_comp == d["cc"].n_comp
        assert ok.status == 0
    L.lsrvt_batch_run([], n_streams=2)


def test_batch_fullsize_64_volumes():
    """The 64-volume batch at full size (edges 32..192, cubes and 2:1:1 boxes,
    3..10 isovalues, T = 15, 8 variables, 32-bin histograms, covariance; 87 M
    voxels) on 4 streams: every job bit-identical to its calls alone; bands
    and components of every job equal the oracle's; cells, sites and site
    components of every job equal the oracle's run of Algorithm 1 (SHA-256
    digests written from the oracle by tests/golden/make_golden.py); cell
    statistics of every job against the oracle's on the (digest-checked)
    labels."""
    from tests import golden_util as G
    from tests.test_gpu_stats import _check_level
    gold, _ = G.load("batch64_t15")
    specs = synth.batch_specs(64, 3)
    data = []
    for shape, seed, k in specs:
        f, iso, w, x, e = synth.fourier_job(shape, seed, k)
        band = oracle.bands(f, iso)
        cc = oracle.components(band, k + 1)
        seeds = synth.seed_sites(cc.comp, cc.n_comp, w, 4096.0, 7919 * seed + 1)
        data.append(dict(f=f, iso=iso, w=w, x=x, edges=e, seeds=seeds, iters=15, cov=True, cc=cc, band=band))
    banner(f"batch full: {len(data)} volumes, {sum(d['f'].size for d in data)} voxels")
    jobs = [L.BatchJob(field=dev(d["f"]), iso=d["iso"], seeds=dev(d["seeds"]), weights=dev(d["w"]), iters=15,
                       variables=dev(d["x"]), edges=dev(d["edges"]), cov=True, cap_comp=int(d["cc"].n_comp) + 16)
            for d in data]
    L.lsrvt_batch_run(jobs, n_streams=4)
    n_oracle = 0
    for i, (d, j) in enumerate(zip(data, jobs)):
        assert j.status == 0 and j.n_comp == d["cc"].n_comp, i
        np.testing.assert_array_equal(host(j.band), d["band"])
        np.testing.assert_array_equal(host(j.comp, np.uint32), d["cc"].comp)
        band, cc, r, st = _alone(d)
        np.testing.assert_array_equal(host(j.cell), host(r.cell))
        S = len(d["seeds"])
        np.testing.assert_array_equal(host(j.sites)[:S], host(r.sites))
        for lvl, (a, b) in enumerate(zip(j.stats, st)):
            units = j.n_comp if lvl == 1 else None
            for key in ("n", "mean", "m2", "vmin", "vmax", "hist", "cov"):
                ga = host(getattr(a, key))
                ga = ga[:units] if units is not None else ga
                assert np.array_equal(ga, host(getattr(b, key))), (i, lvl, key)
        cell = host(j.cell, np.uint32)
        sites = host(j.sites, np.uint32)[:S]
        site_comp = host(j.site_comp, np.uint32)[:S]
        g = gold["jobs"][i]
        assert list(d["f"].shape) == g["shape"] and G.sha(d["seeds"]) == g["seeds_sha256"], f"job {i} inputs"
        G.check_labels(cell, g, f"job {i}")
        assert G.sha(sites) == g["sites_sha256"], f"job {i} sites"
        assert G.sha(site_comp) == g["site_comp_sha256"], f"job {i} site components"
        # the labels are the oracle's (their digest matched): its cell statistics
        _check_level(f"job {i} cells", j.stats[0], oracle.stats(cell, S, d["x"], d["edges"], cov=True), 8)
        n_oracle += 1
    print(f"jobs checked against the oracle's Lloyd loop: {n_oracle} of {len(jobs)}")
