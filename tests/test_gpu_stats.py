"""GPU parity of the statistics rows (Sec. 3.3 "Aggregation", merged up the
hierarchy of Sec. 3.2.4 / Fig. 5) against the oracle's direct FP64 statistics.

Counts, minima, maxima and histograms must match exactly.  Moments use the
tolerances derived from the arithmetic (float32 compensated sums, float64
merges):
  mean:  |mu - mu*|  <= 1e-6 * max(|mu*|, sigma*)
  var:   |v - v*|    <= 1e-5 * v*            (exactly 0 when v* == 0)
  cov:   |c - c*|    <= 1e-5 * sqrt(v*_j v*_k)
where v = M2 / n and c = C_jk / n.  The plain relative error on a mean or a
covariance near zero is not attainable in float32 and is not asserted.
"""
import numpy as np
import pytest

import oracle
import paper_2208_06970_amd as L
import synth
from tests.gpu_util import banner, dev, host

pytestmark = pytest.mark.gpu
NONE = oracle.NONE_ID


def _pairs(m):
    return [(j, k) for j in range(m) for k in range(j, m)]


def _check_level(name, got, want, m, exact_only=False, fp64=False):
    n = host(got.n).astype(np.uint64)
    np.testing.assert_array_equal(n, want.n, err_msg=f"{name} n")
    np.testing.assert_array_equal(host(got.vmin), want.vmin, err_msg=f"{name} min")
    np.testing.assert_array_equal(host(got.vmax), want.vmax, err_msg=f"{name} max")
    if want.hist is not None:
        np.testing.assert_array_equal(host(got.hist, np.uint32), want.hist, err_msg=f"{name} hist")
    nz = want.n > 0
    nn = np.maximum(want.n, 1).astype(np.float64)
    var_w = want.m2 / nn[:, None]
    sd_w = np.sqrt(var_w)
    mean = host(got.mean).astype(np.float64)
    err = np.abs(mean - want.mean)[nz]
    bound = 1e-6 * np.maximum(np.abs(want.mean), sd_w)[nz]
    assert np.all(err <= bound + 0.0), f"{name} mean: worst {np.max(err / np.maximum(bound, 1e-300))}"
    var_g = host(got.m2).astype(np.float64) / nn[:, None]
    verr = np.abs(var_g - var_w)[nz]
    vb = 1e-5 * var_w[nz]
    assert np.all(verr <= vb), f"{name} var: worst ratio {np.max(verr / np.maximum(vb, 1e-300))}"
    assert np.all(host(got.mean)[~nz] == 0) and np.all(host(got.m2)[~nz] == 0)
    worst = {"mean": _ratio(err, bound), "var": _ratio(verr, vb)}
    lit = {"mean": _rel(mean[nz], want.mean[nz]), "var": _rel(var_g[nz], var_w[nz])}
    if want.cov is not None:
        cg = host(got.cov).astype(np.float64) / nn[:, None]
        cw = want.cov / nn[:, None]
        worst["cov"] = lit["cov"] = 0.0
        for p, (j, k) in enumerate(_pairs(m)):
            b = 1e-5 * np.sqrt(var_w[:, j] * var_w[:, k])
            e = np.abs(cg[:, p] - cw[:, p])
            assert np.all(e[nz] <= b[nz]), f"{name} cov({j},{k}): worst {np.max(e[nz] / np.maximum(b[nz], 1e-300))}"
            worst["cov"] = max(worst["cov"], _ratio(e[nz], b[nz]))
            lit["cov"] = max(lit["cov"], _rel(cg[nz, p], cw[nz, p]))
    # worst error as a fraction of the tolerance, and the plain relative error
    print(f"[precision] {name}: of tolerance " + " ".join(f"{k} {v:.3g}" for k, v in worst.items())
          + "; relative " + " ".join(f"{k} {v:.3g}" for k, v in lit.items()), flush=True)
    return True


def _ratio(err, bound):
    """Largest err / bound (0 where both are 0)."""
    if err.size == 0:
        return 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(bound > 0, err / np.where(bound > 0, bound, 1.0), np.where(err > 0, np.inf, 0.0))
    return float(np.max(r))


def _rel(got, want):
    """Largest |got - want| / |want| over the entries with want != 0."""
    m = want != 0
    if not np.any(m):
        return 0.0
    return float(np.max(np.abs(got[m] - want[m]) / np.abs(want[m])))


def _run(shape, seed, m, B, cov, T=3, kind="fourier", rho=128.0, drop_comp_seeds=False, var_gen=None):
    if kind == "blobs":
        wl = synth.blobs_workload(shape, seed, T)
        f, iso, w = wl.field, wl.iso, None
        variables = wl.variables[:m]
        edges = wl.edges[:m] if B else None
    else:
        f = synth.fourier_field(shape, seed, n_modes=96, kmax=max(2.0, min(shape) / 6))
        iso = synth.quantile_isovalues(f, [0.3, 0.55, 0.8])
        w = synth.gradient_weight(f)
        variables = var_gen(shape, m, seed) if var_gen else np.stack(
            [synth.fourier_field(shape, 100 * seed + j, n_modes=64, kmax=8) * (1 + j) + 10.0 * j for j in range(m)])
        edges = synth.histogram_edges(variables, B) if B else None
    band = oracle.bands(f, iso)
    cc = oracle.components(band, len(iso) + 1)
    seeds = synth.seed_sites(cc.comp, cc.n_comp, w, rho, seed)
    if drop_comp_seeds:     # leave some components without sites: their voxels are NONE
        keep = cc.comp.ravel()[seeds] % 5 != 1
        seeds = seeds[keep]
    r = oracle.cvt(cc.comp, seeds, w, T)
    S = len(seeds)
    banner(f"aggregate shape={shape} m={m} B={B} cov={cov} S={S} comps={cc.n_comp}")
    got = L.lsrvt_aggregate(dev(r.cell), dev(r.sites), dev(r.site_comp), dev(cc.comp_band), cc.n_comp,
                            len(iso) + 1, dev(variables.astype(np.float32)),
                            None if edges is None else dev(edges), cov=cov)
    cell_w = oracle.stats(r.cell, S, variables, edges, cov)
    comp_unit = np.where(r.cell == NONE, NONE, r.site_comp[np.minimum(r.cell, max(S - 1, 0))]).astype(np.uint32)
    comp_w = oracle.stats(comp_unit, cc.n_comp, variables, edges, cov)
    band_unit = np.where(r.cell == NONE, NONE, band.astype(np.uint32))
    band_w = oracle.stats(band_unit, len(iso) + 1, variables, edges, cov)
    _check_level("cell", got[0], cell_w, m)
    _check_level("comp", got[1], comp_w, m, fp64=True)
    _check_level("band", got[2], band_w, m, fp64=True)
    return got, (cell_w, comp_w, band_w)


def test_stats_blobs_64():
    _run((64, 64, 64), 1, 3, 16, False, T=10, kind="blobs", rho=512.0)


def test_stats_fourier_cov8_ragged():
    _run((37, 45, 52), 2, 8, 32, True)


def test_stats_many_vars_cov():
    _run((30, 26, 41), 3, 18, 32, True, rho=300.0)        # 189 units: one lane each


def test_stats_units_beyond_lanes():
    _run((22, 27, 19), 4, 24, 8, True, rho=200.0)         # 324 units: two slots per lane


def test_stats_giant_cells_and_unseeded_components():
    # few sites: cells span many box rows and work items; some components unseeded
    _run((48, 64, 70), 5, 4, 16, True, rho=40000.0, drop_comp_seeds=True)


def test_stats_offsets_and_constant_variable():
    def gen(shape, m, seed):
        rng = np.random.default_rng(seed)
        a = 1000.0 + rng.normal(0.0, 0.01, size=shape)      # mean >> sigma
        b = np.full(shape, 3.25)                            # constant: variance exactly 0
        c = rng.normal(0.0, 1.0, size=shape)                # mean ~ 0
        return np.stack([a, b, c]).astype(np.float32)
    got, want = _run((33, 34, 35), 6, 3, 12, True, var_gen=gen)
    for lvl in got:
        nz = host(lvl.n) > 0
        assert np.all(host(lvl.m2)[nz, 1] == 0.0)


def test_stats_without_hist_and_determinism():
    f = synth.fourier_field((40, 41, 42), 7, n_modes=64, kmax=6)
    iso = synth.quantile_isovalues(f, [0.5])
    band = oracle.bands(f, iso)
    cc = oracle.components(band, 2)
    seeds = synth.seed_sites(cc.comp, cc.n_comp, None, 200.0, 7)
    r = oracle.cvt(cc.comp, seeds, None, 2)
    x = np.stack([f, f * f]).astype(np.float32)
    args = (dev(r.cell), dev(r.sites), dev(r.site_comp), dev(cc.comp_band), cc.n_comp, 2, dev(x))
    banner("aggregate determinism")
    a = L.lsrvt_aggregate(*args, None, cov=True)
    b = L.lsrvt_aggregate(*args, None, cov=True)
    for la, lb in zip(a, b):
        for k in ("n", "mean", "m2", "vmin", "vmax", "cov"):
            assert np.array_equal(host(getattr(la, k)), host(getattr(lb, k))), k
    _check_level("cell", a[0], oracle.stats(r.cell, len(seeds), x, None, True), 2)


@pytest.mark.parametrize("tile", [1, 2, 4])
def test_stats_every_staging_tile(tile):
    """Each statistics tile the autotuner may choose (voxels per thread and
    staging round) stays within the tolerances; giant cells so that every
    item spans several rounds."""
    prev = L.lsrvt_set_tuning(L.TUNE_STATS_TILE, tile)
    try:
        _run((40, 44, 52), 6, 18, 32, True, rho=6000.0)
    finally:
        L.lsrvt_set_tuning(L.TUNE_STATS_TILE, prev)
