"""Joint moments up to fourth order (lsrvt_comoments) against the oracle's
direct two-pass float64 sums, per cell, component and band.

Tolerance: every sum is float64; a cell's thread sums at most n products in
order (error below n u sum|terms|, n <= 2^20 here, u = 2^-53) and the
merges are the stable pairwise formulas, so entries are compared to
1e-8 x the natural scale n sigma_i sigma_j ... of the entry (sigma from the
oracle's M2), means to 1e-10 x max(|mean|, sigma).  Units with no voxels
must be exactly zero."""
import numpy as np
import pytest

import oracle
import paper_2208_06970_amd as L
import synth
from tests.gpu_util import banner, dev, host

pytestmark = pytest.mark.gpu
NONE = oracle.NONE_ID


def _scale(mo, m):
    n = mo.n.astype(np.float64)
    t2 = oracle.tuples(m, 2)
    var = np.stack([mo.m2[:, t2.index((j, j))] for j in range(m)], axis=1)
    sig = np.sqrt(np.maximum(var, 0) / np.maximum(n, 1)[:, None])
    out = []
    for r in (2, 3, 4):
        tups = oracle.tuples(m, r)
        s = np.stack([np.prod(sig[:, list(t)], axis=1) for t in tups], axis=1) * n[:, None]
        out.append(s)
    return sig, out


def _check(name, got, want, m):
    gn = host(got.n).astype(np.uint64)
    np.testing.assert_array_equal(gn, want.n, err_msg=f"{name} n")
    sig, scales = _scale(want, m)
    gmean = host(got.mean)
    tol_mean = 1e-10 * np.maximum(np.abs(want.mean), sig) + 1e-300
    assert np.all(np.abs(gmean - want.mean) <= tol_mean), f"{name} mean"
    worst = 0.0
    for key, sc in zip(("m2", "m3", "m4"), scales):
        g = host(getattr(got, key))
        w = getattr(want, key)
        err = np.abs(g - w)
        empty = want.n == 0
        assert np.all(g[empty] == 0), f"{name} {key} of empty units"
        ok = err <= 1e-8 * sc + 1e-300
        assert np.all(ok | empty[:, None]), f"{name} {key}: worst {np.max(err / np.maximum(sc, 1e-300))}"
        worst = max(worst, float(np.max((err / np.maximum(sc, 1e-300))[~empty])) if np.any(~empty) else 0.0)
    return worst


def _case(shape, seed, n_iso, m, iters, rho):
    f = synth.fourier_field(shape, seed, n_modes=64)
    iso = synth.quantile_isovalues(f, [(i + 1) / (n_iso + 1) for i in range(n_iso)])
    w = synth.gradient_weight(f)
    x = np.stack([synth.fourier_field(shape, 50 * seed + j, n_modes=64) for j in range(m)]).astype(np.float32)
    x[0] = x[0] ** 3  # a skewed variable
    band = oracle.bands(f, iso)
    cc = oracle.components(band, n_iso + 1)
    seeds = synth.seed_sites(cc.comp, cc.n_comp, w, rho, seed)
    b = dev(band)
    g = L.lsrvt_components(b, n_iso + 1)
    r = L.lsrvt_cvt(b, g.comp, dev(seeds), dev(w), iters, want_mean_ds=False)
    return x, cc, g, r, n_iso + 1


def _units(cell, site_comp, comp_band):
    c = cell.ravel()
    lab = c != NONE
    comp = np.full(c.shape, NONE, dtype=np.uint32)
    comp[lab] = site_comp[c[lab]]
    bnd = np.full(c.shape, NONE, dtype=np.uint32)
    bnd[lab] = comp_band[comp[lab]]
    return c, comp, bnd


@pytest.mark.parametrize("shape,seed,n_iso,m,iters,rho", [
    ((40, 36, 44), 1, 3, 4, 2, 200.0),
    ((33, 48, 29), 2, 5, 8, 1, 120.0),
    ((20, 64, 24), 3, 2, 1, 3, 400.0),
    ((28, 20, 36), 5, 4, 13, 2, 150.0),   # 13 variables: two passes of the cell sums
    ((24, 30, 20), 6, 3, 18, 1, 300.0),   # 18 variables (the combustion workload's count)
])
def test_comoments_match_oracle(shape, seed, n_iso, m, iters, rho):
    x, cc, g, r, nb = _case(shape, seed, n_iso, m, iters, rho)
    banner(f"comoments: {shape} m={m}")
    cm, gm, bm = L.lsrvt_comoments(r.cell, r.sites, r.site_comp, g.comp_band, g.n_comp, nb, dev(x))
    cell = host(r.cell, np.uint32)
    sc = host(r.site_comp, np.uint32)
    cb = host(g.comp_band).astype(np.uint32)
    uc, ug, ub = _units(cell, sc, cb)
    S = int(r.sites.numel())
    w1 = _check("cell", cm, oracle.comoments(uc, S, x), m)
    w2 = _check("comp", gm, oracle.comoments(ug, g.n_comp, x), m)
    w3 = _check("band", bm, oracle.comoments(ub, nb, x), m)
    print(f"worst relative errors: cell {w1:.2e} comp {w2:.2e} band {w3:.2e}")


def test_comoments_empty_cells_and_determinism():
    x, cc, g, r, nb = _case((24, 24, 24), 4, 3, 3, 1, 64.0)
    banner("comoments: determinism")
    a = L.lsrvt_comoments(r.cell, r.sites, r.site_comp, g.comp_band, g.n_comp, nb, dev(x))
    b = L.lsrvt_comoments(r.cell, r.sites, r.site_comp, g.comp_band, g.n_comp, nb, dev(x))
    for p, q in zip(a, b):
        for k in ("n", "mean", "m2", "m3", "m4"):
            assert np.array_equal(host(getattr(p, k)), host(getattr(q, k))), k
    # all voxels unlabelled: every unit is empty
    none = dev(np.full(x.shape[1:], NONE, dtype=np.uint32))
    cm, gm, bm = L.lsrvt_comoments(none, r.sites, r.site_comp, g.comp_band, g.n_comp, nb, dev(x))
    for mo in (cm, gm, bm):
        assert np.all(host(mo.n) == 0)
        for k in ("mean", "m2", "m3", "m4"):
            assert np.all(host(getattr(mo, k)) == 0), k


def test_comoments_fullsize_sampled():
    """The 256^3 benchmark cells (T = 20 loop, 8 variables): a sample of cells
    and of components against the oracle on their voxels, and the band level
    of the first four variables over the whole volume."""
    wl = synth.fourier_workload()
    band = oracle.bands(wl.field, wl.iso)
    cc = oracle.components(band, wl.n_bands)
    seeds = synth.workload_sites(wl, cc.comp, cc.n_comp)
    b = dev(band)
    g = L.lsrvt_components(b, wl.n_bands)
    banner("comoments: 256^3 Lloyd loop")
    r = L.lsrvt_cvt(b, g.comp, dev(seeds), dev(wl.weights), wl.iters, want_mean_ds=False)
    x = np.ascontiguousarray(wl.variables)
    banner("comoments: 256^3, 8 variables")
    cm, gm, bm = L.lsrvt_comoments(r.cell, r.sites, r.site_comp, g.comp_band, g.n_comp, wl.n_bands, dev(x))
    cell = host(r.cell, np.uint32).ravel()
    sc = host(r.site_comp, np.uint32)
    cb = host(g.comp_band).astype(np.uint32)
    uc, ug, ub = _units(cell, sc, cb)
    S = len(seeds)
    rng = np.random.default_rng(0)
    counts = np.bincount(uc[uc != NONE], minlength=S)
    pick_c = np.unique(np.concatenate([np.argsort(-counts)[:10], rng.choice(S, 200, replace=False)]))
    sel = np.isin(uc, pick_c)
    want = oracle.comoments(uc[sel], S, x.reshape(8, -1)[:, sel])
    keep = np.zeros(S, dtype=bool)
    keep[pick_c] = True
    sub = lambda mo, k: L.Moments(mo.n[k], mo.mean[k], mo.m2[k], mo.m3[k], mo.m4[k])
    idx = dev(np.flatnonzero(keep).astype(np.int64))
    wsub = oracle.Moments(want.n[keep], want.mean[keep], want.m2[keep], want.m3[keep], want.m4[keep])
    _check("cell sample", sub(cm, idx), wsub, 8)
    compn = np.bincount(ug[ug != NONE], minlength=g.n_comp)
    pick_g = np.unique(np.concatenate([np.argsort(-compn)[:5], rng.choice(g.n_comp, 200, replace=False)]))
    sel = np.isin(ug, pick_g)
    want = oracle.comoments(ug[sel], g.n_comp, x.reshape(8, -1)[:, sel])
    keep = np.zeros(g.n_comp, dtype=bool)
    keep[pick_g] = True
    idx = dev(np.flatnonzero(keep).astype(np.int64))
    wsub = oracle.Moments(want.n[keep], want.mean[keep], want.m2[keep], want.m3[keep], want.m4[keep])
    _check("comp sample", sub(gm, idx), wsub, 8)
    banner("comoments: 256^3 bands, 4 variables")
    x4 = np.ascontiguousarray(x[:4])
    cm4, gm4, bm4 = L.lsrvt_comoments(r.cell, r.sites, r.site_comp, g.comp_band, g.n_comp, wl.n_bands, dev(x4))
    _check("band", bm4, oracle.comoments(ub, wl.n_bands, x4), 4)
