"""The combustion-shaped workload: a thin wrinkled flame sheet, 1024 x 512 x 512
voxels (nx, ny, nz), 10 isovalues of the mixture fraction, |grad T| weights,
30 updates, 18 variables (Z, T, 16 species) with 32-bin histograms and the
full 18 x 18 covariance.

* A 128 x 64 x 64 box of the same generator is checked whole against the
  oracle: labels, cells and sites bit-exact, statistics of every cell,
  component and band within the tolerances of the statistics tests.
* At full size (2^28 voxels) bands and components are compared element by
  element over the whole volume.  Cells and sites after 30 updates are
  compared bit for bit on a sample of the components whose bounding box holds
  at most 2^18 voxels, each cropped to its
  bounding box: the crop keeps the order of linear indices and of site ids,
  so every tie breaks as in the whole volume.  The largest components are
  checked through one update (the oracle's update of sampled cells of the
  29-update run must give the 30-update run's sites) and properties that hold
  at any size (each labelled voxel's cell is a site of its component, sampled
  cells are 6-connected and hold their site).  Statistics: sampled cells and
  components against the oracle on their crops; every component's and band's
  voxel count exactly.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
import paper_2208_06970_amd as L
import synth
from tests.gpu_util import banner, dev, host
from tests.test_gpu_stats import _check_level

pytestmark = pytest.mark.gpu
NONE = oracle.NONE_ID
SIX = ndimage.generate_binary_structure(3, 1)


def _sub(level, idx):
    """Rows idx of a LevelStats (device tensors), for _check_level."""
    return L.LevelStats(*(None if getattr(level, k) is None else getattr(level, k)[idx]
                          for k in ("n", "mean", "m2", "vmin", "vmax", "hist", "cov")))


def test_flame_small_whole_volume():
    wl = synth.flame_workload(shape=(64, 64, 128))
    band = oracle.bands(wl.field, wl.iso)
    cc = oracle.components(band, wl.n_bands)
    seeds = synth.flame_sites(cc.comp, cc.n_comp, wl.weights, 512.0, wl.seed)
    banner(f"flame 128x64x64: comps={cc.n_comp} sites={len(seeds)}")
    b, st = L.lsrvt_isobands(dev(wl.field), wl.iso)
    np.testing.assert_array_equal(host(b), band)
    g = L.lsrvt_components(b, wl.n_bands)
    assert g.n_comp == cc.n_comp
    np.testing.assert_array_equal(host(g.comp, np.uint32), cc.comp)
    r = L.lsrvt_cvt(b, g.comp, dev(seeds), dev(wl.weights), wl.iters)
    want = oracle.cvt(cc.comp, seeds, wl.weights, wl.iters)
    np.testing.assert_array_equal(host(r.sites, np.uint32), want.sites)
    np.testing.assert_array_equal(host(r.cell, np.uint32), want.cell)
    np.testing.assert_allclose(r.mean_ds, want.mean_ds, rtol=1e-12, atol=0)
    banner("flame 128x64x64: statistics, 18 variables, covariance")
    x = np.ascontiguousarray(wl.variables)
    cs, gs, bs = L.lsrvt_aggregate(r.cell, r.sites, r.site_comp, g.comp_band, g.n_comp, wl.n_bands, dev(x),
                                   dev(wl.edges), cov=True)
    S = len(seeds)
    _check_level("cell", cs, oracle.stats(want.cell, S, x, wl.edges, cov=True), 18)
    cu = np.where(want.cell == NONE, NONE, want.site_comp[np.minimum(want.cell, S - 1)]).astype(np.uint32)
    _check_level("comp", gs, oracle.stats(cu, cc.n_comp, x, wl.edges, cov=True), 18)
    bu = np.where(want.cell == NONE, NONE, band.astype(np.uint32))
    _check_level("band", bs, oracle.stats(bu, wl.n_bands, x, wl.edges, cov=True), 18)


def test_flame_fullsize_sampled():
    banner("flame 1024x512x512: generating")
    wl = synth.flame_workload()
    nz, ny, nx = wl.shape
    band = oracle.bands(wl.field, wl.iso)
    banner("flame full: isobands")
    b, st = L.lsrvt_isobands(dev(wl.field), wl.iso)
    assert int(host(st)[0]) == 0
    np.testing.assert_array_equal(host(b), band)
    cc = oracle.components(band, wl.n_bands)
    banner(f"flame full: components ({cc.n_comp})")
    g = L.lsrvt_components(b, wl.n_bands)
    assert g.n_comp == cc.n_comp
    np.testing.assert_array_equal(host(g.comp, np.uint32), cc.comp)
    np.testing.assert_array_equal(host(g.comp_band), cc.comp_band)
    seeds = synth.flame_sites(cc.comp, cc.n_comp, wl.weights, wl.rho, wl.seed)
    S = len(seeds)
    T = wl.iters
    banner(f"flame full: Lloyd loops of {T - 1} and {T} updates, S={S}")
    d_w, d_seeds = dev(wl.weights), dev(seeds)
    r0 = L.lsrvt_cvt(b, g.comp, d_seeds, d_w, T - 1, want_mean_ds=False)
    cell0 = host(r0.cell, np.uint32)
    sites0 = host(r0.sites, np.uint32)
    del r0
    r = L.lsrvt_cvt(b, g.comp, d_seeds, d_w, T, want_mean_ds=False)
    cell = host(r.cell, np.uint32)
    sites = host(r.sites, np.uint32)
    site_comp = host(r.site_comp, np.uint32)
    comp = cc.comp
    cflat = cell.ravel()
    # every labelled voxel's cell is a site of its own component; exactly the
    # components without a site stay unlabelled
    lab = cflat != NONE
    np.testing.assert_array_equal(site_comp[cflat[lab]], comp.ravel()[lab])
    seeded = np.zeros(cc.n_comp, dtype=bool)
    seeded[site_comp] = True
    np.testing.assert_array_equal(lab, seeded[comp.ravel()])
    del lab

    boxes = ndimage.find_objects(comp.astype(np.int32) + 1)
    vol = np.array([np.prod([s.stop - s.start for s in bx]) for bx in boxes])
    rng = np.random.default_rng(11)
    small = np.flatnonzero(seeded & (vol <= (1 << 18)))
    pick = rng.choice(small, min(30, len(small)), replace=False) if len(small) else []
    x = wl.variables
    checked = 0
    for c in pick:
        bx = boxes[c]
        crop = comp[bx] == c
        ids = np.flatnonzero(site_comp == c)               # global ids, in order
        lo = np.array([s.start for s in bx])
        shp = crop.shape
        def local(v):
            v = v.astype(np.int64)
            zz, yy, xx = v // (nx * ny) - lo[0], (v // nx) % ny - lo[1], v % nx - lo[2]
            return ((zz * shp[1] + yy) * shp[2] + xx).astype(np.uint32)
        ccrop = np.where(crop, 0, NONE).astype(np.uint32)
        want = oracle.cvt(ccrop, local(seeds[ids]), wl.weights[bx], T)
        got_cell = cell[bx]
        exp_cell = np.where(crop, ids[np.minimum(want.cell, len(ids) - 1)], NONE)
        np.testing.assert_array_equal(np.where(crop, got_cell, NONE), exp_cell, err_msg=f"component {c}")
        np.testing.assert_array_equal(local(sites[ids]), want.sites, err_msg=f"component {c} sites")
        checked += 1
    print(f"components cropped and compared: {checked} of {int(seeded.sum())} seeded")

    # the largest components: one update per sampled cell, and connected cells
    big = np.flatnonzero(seeded & (vol > (1 << 18)))
    big_sites = np.flatnonzero(np.isin(site_comp, big))
    samp = rng.choice(big_sites, min(24, len(big_sites)), replace=False) if len(big_sites) else []
    for s in samp:
        for lbl, cl in ((0, cell0), (1, cell)):
            m = cl == s
            if not m.any():
                continue
            bx = ndimage.find_objects(m.astype(np.int8))[0]
            mm = m[bx]
            if lbl == 0:
                lo = np.array([t.start for t in bx])
                shp = mm.shape
                v0 = int(sites0[s])
                p0 = np.array([v0 // (nx * ny), (v0 // nx) % ny, v0 % nx]) - lo
                # the old position matters only for an empty cell (weights >= 1 here)
                l0 = int((p0[0] * shp[1] + p0[1]) * shp[2] + p0[2]) if np.all((p0 >= 0) & (p0 < shp)) else 0
                new, _ = oracle.update(np.where(mm, 0, NONE).astype(np.uint32), [l0], wl.weights[bx])
                q = int(new[0])
                gz, gy, gx = q // (shp[1] * shp[2]) + lo[0], (q // shp[2]) % shp[1] + lo[1], q % shp[2] + lo[2]
                assert int(sites[s]) == (gz * ny + gy) * nx + gx, f"site {s}: one update"
            else:
                _, k = ndimage.label(mm, structure=SIX)
                assert k == 1, f"cell {s} is not 6-connected"
                v = int(sites[s])
                assert cflat[v] == s or sites[cflat[v]] == v

    banner("flame full: statistics, 18 variables, covariance")
    cs, gs, bs = L.lsrvt_aggregate(r.cell, r.sites, r.site_comp, g.comp_band, g.n_comp, wl.n_bands, dev(x),
                                   dev(wl.edges), cov=True)
    del r
    n_b = np.bincount(band.ravel()[cflat != NONE], minlength=wl.n_bands)
    np.testing.assert_array_equal(host(bs.n).astype(np.int64), n_b)
    n_c = np.bincount(site_comp[cflat[cflat != NONE]], minlength=cc.n_comp)
    np.testing.assert_array_equal(host(gs.n).astype(np.int64), n_c)
    # sampled cells (both kinds) and sampled small components on their crops
    cells = np.unique(np.concatenate([np.asarray(samp, dtype=np.int64),
                                      rng.choice(S, 40, replace=False).astype(np.int64)]))
    for s in cells:
        m = cell == s
        if not m.any():
            continue
        bx = ndimage.find_objects(m.astype(np.int8))[0]
        unit = np.where(m[bx], 0, NONE).astype(np.uint32)
        xs = np.ascontiguousarray(x[(slice(None),) + bx])
        want = oracle.stats(unit, 1, xs, wl.edges, cov=True)
        _check_level(f"cell {s}", _sub(cs, [s]), want, 18)
    for c in pick[:10]:
        bx = boxes[c]
        unit = np.where((comp[bx] == c) & (cell[bx] != NONE), 0, NONE).astype(np.uint32)
        xs = np.ascontiguousarray(x[(slice(None),) + bx])
        want = oracle.stats(unit, 1, xs, wl.edges, cov=True)
        _check_level(f"component {c}", _sub(gs, [c]), want, 18)


def test_flame_fullsize_against_oracle():
    """The whole 2^28-voxel Lloyd loop (30 updates) bit for bit against the
    oracle's run of Algorithm 1 on the same inputs, through the digests
    ``tests/golden/make_golden.py`` stored (cells, sites, site components, and
    the cells of every component to name the first one that differs), and
    the statistics of components and bands against the oracle's stored ones:
    exact digests of counts, extrema and histograms, moments and covariance
    within the tolerances of the statistics tests."""
    from tests import golden_util as G
    doc, arrays = G.load("flame_t30")
    banner("flame golden: generating 1024x512x512")
    wl = synth.flame_workload()
    b, _ = L.lsrvt_isobands(dev(wl.field), wl.iso)
    g = L.lsrvt_components(b, wl.n_bands)
    assert g.n_comp == doc["n_comp"]
    comp = host(g.comp, np.uint32)
    seeds = synth.flame_sites(comp, g.n_comp, wl.weights, wl.rho, wl.seed)
    assert G.sha(seeds) == doc["seeds_sha256"], "inputs differ from the ones the oracle ran on"
    banner(f"flame golden: Lloyd loop, {wl.iters} updates, S={len(seeds)}")
    r = L.lsrvt_cvt(b, g.comp, dev(seeds), dev(wl.weights), wl.iters)
    cell = host(r.cell, np.uint32)
    if G.sha(cell) != doc["cell_sha256"]:
        kflat, cflat = comp.ravel(), cell.ravel()
        order = np.argsort(kflat, kind="stable")
        bounds = np.searchsorted(kflat[order], np.arange(g.n_comp + 1))
        for c in range(g.n_comp):
            if G.sha(cflat[order[bounds[c]:bounds[c + 1]]]) != doc["comp_cell_sha256"][c]:
                raise AssertionError(f"flame T=30 cells differ from the oracle's, first in component {c}")
        G.check_labels(cell, doc, "flame T=30")
    assert G.sha(host(r.sites, np.uint32)) == doc["sites_sha256"]
    assert G.sha(host(r.site_comp, np.uint32)) == doc["site_comp_sha256"]
    np.testing.assert_allclose(r.mean_ds, doc["mean_ds"], rtol=1e-12, atol=0)
    del cell
    banner("flame golden: statistics of components and bands, 18 variables, covariance")
    x = dev(np.ascontiguousarray(wl.variables))
    cs, gs, bs = L.lsrvt_aggregate(r.cell, r.sites, r.site_comp, g.comp_band, g.n_comp, wl.n_bands, x,
                                   dev(wl.edges), cov=True)
    G.exact_digests_match(gs, doc["comp_exact_sha256"], "component")
    G.exact_digests_match(bs, doc["band_exact_sha256"], "band")
    rows = arrays["comp_rows"]
    _check_level("component", _sub(gs, rows), G.level_stats(arrays, "comp"), 18)
    _check_level("band", bs, G.level_stats(arrays, "band"), 18)
