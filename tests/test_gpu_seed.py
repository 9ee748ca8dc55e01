"""Stratified initial sites on the GPU (lsrvt_seed) against the oracle:
exact equality of the site list (every decision is integer arithmetic), on
volumes that span several blocks with ragged edges, with and without weights
and mass tables, in the degenerate cases (zero-mass components, a block full
of one-voxel components, volumes smaller than a block, capacity retries), and
on the 256^3 benchmark field through properties that hold at any size."""
import math

import numpy as np
import pytest

import oracle
import paper_2208_06970_amd as L
import synth
from oracle import seeding
from tests import brute
from tests.gpu_util import banner, dev, host

pytestmark = pytest.mark.gpu


def _gpu(comp, cc, w=None, lut=None, **kw):
    first = cc.comp_first.astype(np.uint32)
    s = L.lsrvt_seed(dev(comp.astype(np.uint32)), dev(first), cc.n_comp,
                     None if w is None else dev(w), None if lut is None else dev(lut), **kw)
    return host(s, np.uint32)


def _field_case(shape, seed, n_iso):
    f = synth.fourier_field(shape, seed, n_modes=48)
    iso = synth.quantile_isovalues(f, [(i + 1) / (n_iso + 1) for i in range(n_iso)])
    band = oracle.bands(f, iso)
    cc = oracle.components(band, n_iso + 1)
    return f, cc


@pytest.mark.parametrize("shape,seed,n_iso,block,rho,weighted", [
    ((40, 37, 45), 1, 3, 16, 300, True),
    ((33, 50, 29), 2, 5, 8, 97, True),
    ((64, 64, 64), 3, 4, 16, 512, False),
    ((17, 70, 23), 4, 2, 4, 40, True),
    ((48, 16, 80), 5, 7, 10, 150, True),
])
def test_seed_matches_oracle(shape, seed, n_iso, block, rho, weighted):
    f, cc = _field_case(shape, seed, n_iso)
    w = synth.gradient_weight(f) if weighted else None
    key = 0x9E3779B97F4A7C15 ^ seed
    banner(f"seed: {shape} block {block} rho {rho} weighted {weighted}")
    got = _gpu(cc.comp, cc, w, None, rho=rho, block=block, seed=key)
    want = oracle.seed_stratified(cc.comp, cc.n_comp, w, None, rho=rho, block=block, seed=key)
    np.testing.assert_array_equal(got, want)


def test_seed_mass_table_and_zero_mass_components():
    f, cc = _field_case((36, 44, 40), 7, 4)
    w = synth.gradient_weight(f)
    # attraction gamma = 0.5 as a table, and a threshold that leaves some components without mass
    lut = np.round(64.0 * np.sqrt(np.arange(65536, dtype=np.float64))).astype(np.uint32)
    cut = lut.copy()
    cut[:np.percentile(w, 60).astype(int)] = 0
    for name, table in (("sqrt", lut), ("cut", cut)):
        banner(f"seed: mass table {name}")
        got = _gpu(cc.comp, cc, w, table, rho=200, block=16, seed=5)
        want = oracle.seed_stratified(cc.comp, cc.n_comp, w, table, rho=200, block=16, seed=5)
        np.testing.assert_array_equal(got, want)
    m = cut[w.ravel()]
    zero = [c for c in range(cc.n_comp) if m[cc.comp.ravel() == c].sum() == 0]
    assert zero, "the cut table should leave components without mass"


def test_seed_degenerate_cases():
    # every voxel its own component (2-band checkerboard): a 16^3 block holds 4096 components
    z, y, x = np.meshgrid(np.arange(20), np.arange(18), np.arange(17), indexing="ij")
    band = ((x + y + z) % 2).astype(np.uint8)
    cc = oracle.components(band, 2)
    assert cc.n_comp == band.size
    banner("seed: checkerboard")
    got = _gpu(cc.comp, cc, None, None, rho=3, block=16, seed=11)
    np.testing.assert_array_equal(got, oracle.seed_stratified(cc.comp, cc.n_comp, None, None, rho=3, block=16,
                                                              seed=11))
    # one component, volume smaller than a block, a single voxel
    for shape in ((5, 3, 7), (1, 1, 1), (1, 1, 40)):
        band = np.zeros(shape, dtype=np.uint8)
        cc = oracle.components(band, 1)
        rng = np.random.default_rng(3)
        w = rng.integers(0, 50, size=shape).astype(np.uint16)
        banner(f"seed: single component {shape}")
        got = _gpu(cc.comp, cc, w, None, rho=2, block=16, seed=1)
        np.testing.assert_array_equal(got, oracle.seed_stratified(cc.comp, cc.n_comp, w, None, rho=2, block=16,
                                                                  seed=1))
    # all weights zero: every component gets its first voxel
    _, cc = _field_case((24, 24, 24), 9, 3)
    zeros = np.zeros(cc.comp.shape, dtype=np.uint16)
    banner("seed: zero weights")
    got = _gpu(cc.comp, cc, zeros, None, rho=10, block=8, seed=2)
    np.testing.assert_array_equal(got, cc.comp_first.astype(np.uint32))


def test_seed_capacity_retry_and_validation():
    _, cc = _field_case((30, 30, 30), 12, 3)
    banner("seed: capacity retries")
    got = _gpu(cc.comp, cc, None, None, rho=20, block=8, seed=4, cap_pairs=1, cap_sites=1)
    np.testing.assert_array_equal(got, oracle.seed_stratified(cc.comp, cc.n_comp, None, None, rho=20, block=8,
                                                              seed=4))
    bad = cc.comp.copy()
    bad.ravel()[5] = cc.n_comp + 3
    with pytest.raises(L.LsrvtError) as e:
        _gpu(bad, cc, None, None, rho=20, block=8, seed=4)
    assert e.value.code == L.EINVAL


def test_seed_fullsize_properties():
    """The 256^3 benchmark field: site counts per component (exact, Eq. 3),
    numbering by (component, block), sites inside their component, pair
    shares against the largest-remainder rule on a sample of components, and
    the oracle's own placement on a sample of pairs."""
    wl = synth.fourier_workload()
    band = oracle.bands(wl.field, wl.iso)
    cc = oracle.components(band, wl.n_bands)
    comp = cc.comp.ravel()
    key, rho, block = 0x5EED, 4096, 16
    banner("seed: 256^3 benchmark field")
    s = _gpu(cc.comp, cc, wl.weights, None, rho=rho, block=block, seed=key)
    s2 = _gpu(cc.comp, cc, wl.weights, None, rho=rho, block=block, seed=key)
    np.testing.assert_array_equal(s, s2)
    m = wl.weights.ravel().astype(np.int64)
    total = int(m.sum())
    n = m.size
    mc = np.bincount(comp, weights=m, minlength=cc.n_comp)  # exact: sums below 2^53
    want_nc = [max(-(-(int(v) * n) // (rho * total)), 1) for v in mc]
    got_nc = np.bincount(comp[s], minlength=cc.n_comp)
    np.testing.assert_array_equal(got_nc, want_nc)
    blk = seeding.block_index(cc.comp.shape, block)
    order = comp[s].astype(np.int64) * (int(blk.max()) + 1) + blk[s]
    assert np.all(np.diff(order) >= 0)
    # a sample of components, shares and placement recomputed by the oracle's steps
    rng = np.random.default_rng(0)
    big = np.argsort(-mc)[:20]
    sample = np.unique(np.concatenate([big, rng.choice(cc.n_comp, 40, replace=False)]))
    for c in sample:
        vox = np.flatnonzero(comp == c)
        pb = blk[vox]
        blocks = np.unique(pb)
        masses = [int(m[vox[pb == b]].sum()) for b in blocks]
        if sum(masses) == 0:
            assert list(s[comp[s] == c]) == [int(vox[0])]
            continue
        shares = seeding.apportion(want_nc[c], masses, blocks)
        mine = s[comp[s] == c]
        for b, mb, nb in zip(blocks, masses, shares):
            here = mine[blk[mine] == b]
            assert len(here) == nb
            if nb:
                pv = vox[pb == b]
                cum = np.cumsum(m[pv])
                o = seeding.pair_offset(key, int(b), int(c), mb)
                exp = [int(pv[np.searchsorted(cum, (o + j * mb) // nb, side="right")]) for j in range(nb)]
                assert list(here) == exp
    assert math.isclose(len(s), sum(want_nc))
