"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test reaches the expected result by a route independent of the oracle
(library routines, brute force, exact rationals, closed forms, invariants), so
a plausible mistake in the oracle -- a dropped term, a wrong sign or index, a
transposed operand, an off-by-one tie rule -- fails at least one of them.
"""
import numpy as np
import pytest

import oracle
from tests import brute

NONE = oracle.NONE_ID


# --------------------------------------------------------------------------
# isobands (Sec. 3.1: B_{a,b} = {a < f <= b})
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bands_match_searchsorted(seed):
    rng = np.random.default_rng(seed)
    iso = np.sort(rng.uniform(-1, 1, size=rng.integers(1, 12))).astype(np.float32)
    iso = np.unique(iso)
    f = rng.uniform(-1.5, 1.5, size=(7, 9, 11)).astype(np.float32)
    # exact ties with isovalues and infinities
    f.ravel()[:len(iso)] = iso
    f.ravel()[-1] = np.inf
    f.ravel()[-2] = -np.inf
    got = oracle.bands(f, iso)
    np.testing.assert_array_equal(got, brute.bands_searchsorted(f, iso))


def test_bands_interval_convention():
    # a value equal to an isovalue belongs to the lower band (a < f <= b)
    iso = np.array([0.0, 1.0], dtype=np.float32)
    f = np.array([-1.0, 0.0, 0.5, 1.0, 2.0], dtype=np.float32).reshape(1, 1, 5)
    np.testing.assert_array_equal(oracle.bands(f, iso).ravel(), [0, 0, 1, 1, 2])


def test_bands_errors():
    f = np.zeros((1, 1, 4), dtype=np.float32)
    with pytest.raises(oracle.OracleError) as e:
        oracle.bands(f, np.array([1.0, 1.0], dtype=np.float32))
    assert e.value.code == oracle.EINVAL
    with pytest.raises(oracle.OracleError) as e:
        oracle.bands(f, np.array([np.nan], dtype=np.float32))
    assert e.value.code == oracle.EINVAL
    f[0, 0, 2] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.bands(f, np.array([0.5], dtype=np.float32))
    assert e.value.code == oracle.ENAN


# --------------------------------------------------------------------------
# connected components (Sec. 3.1), canonical (band, min index) numbering
@pytest.mark.parametrize("shape,n_bands,smooth,seed", [
    ((6, 6, 6), 2, False, 0), ((5, 4, 7), 3, False, 1), ((1, 1, 9), 2, False, 2),
    ((1, 8, 8), 3, False, 3), ((16, 12, 20), 4, True, 4), ((24, 24, 24), 5, True, 5),
    ((30, 1, 30), 3, False, 6),
])
def test_components_match_scipy(shape, n_bands, smooth, seed):
    rng = np.random.default_rng(seed)
    band = brute.random_bands(shape, n_bands, rng, smooth)
    got = oracle.components(band, n_bands)
    comp, k, cb, cs, cf, bo = brute.components_scipy(band, n_bands)
    assert got.n_comp == k
    np.testing.assert_array_equal(got.comp, comp)
    np.testing.assert_array_equal(got.comp_band, cb)
    np.testing.assert_array_equal(got.comp_size, cs)
    np.testing.assert_array_equal(got.comp_first, cf)
    np.testing.assert_array_equal(got.band_offset, bo)


@pytest.mark.parametrize("seed", range(4))
def test_components_match_unionfind(seed):
    rng = np.random.default_rng(100 + seed)
    band = brute.random_bands((4, 5, 6), 2, rng)
    np.testing.assert_array_equal(oracle.components(band, 2).comp, brute.components_unionfind(band))


def test_components_single_band_and_checkerboard():
    band = np.zeros((3, 4, 5), dtype=np.uint8)
    c = oracle.components(band, 1)
    assert c.n_comp == 1 and c.comp_size[0] == 60 and c.comp_first[0] == 0
    z, y, x = np.indices((3, 4, 5))
    cb = ((x + y + z) % 2).astype(np.uint8)
    c = oracle.components(cb, 2)
    assert c.n_comp == 60                      # every voxel isolated
    assert list(c.band_offset) == [0, 30, 60]


# --------------------------------------------------------------------------
# restricted geodesic Voronoi regions (Eq. 1), hop metric, ties to lower id
@pytest.mark.parametrize("shape,n_bands,S,seed", [
    ((4, 4, 4), 2, 5, 0), ((5, 5, 5), 3, 9, 1), ((6, 6, 6), 2, 12, 2), ((1, 1, 12), 2, 4, 3),
    ((1, 7, 9), 2, 6, 4), ((6, 5, 4), 1, 7, 5),
])
def test_vt_matches_allpairs_bruteforce(shape, n_bands, S, seed):
    rng = np.random.default_rng(seed)
    band = brute.random_bands(shape, n_bands, rng, smooth=min(shape) > 3)
    comp = oracle.components(band, n_bands).comp
    n = comp.size
    sites = rng.integers(0, n, size=S).astype(np.uint32)
    sites[-1] = sites[0]                       # a duplicate: the higher id keeps an empty cell
    want_cell, want_dist = brute.vt_allpairs(comp, sites)
    for pruned in (True, False):
        cell, dist = oracle.vt(comp, sites, pruned=pruned, return_dist=True)
        np.testing.assert_array_equal(cell, want_cell)
        fin = want_cell != NONE
        np.testing.assert_array_equal(dist[fin], want_dist[fin].astype(np.uint32))
    assert not np.any(cell == S - 1)


@pytest.mark.parametrize("seed", range(3))
def test_vt_pruned_equals_unpruned_medium(seed):
    rng = np.random.default_rng(50 + seed)
    band = brute.random_bands((14, 15, 16), 3, rng, smooth=True)
    comp = oracle.components(band, 3).comp
    sites = rng.choice(comp.size, size=40, replace=False).astype(np.uint32)
    np.testing.assert_array_equal(oracle.vt(comp, sites, True), oracle.vt(comp, sites, False))


def test_vt_octants_closed_form():
    # uniform 10^3 block, 8 seeds at {2,7}^3: the regions are the 8 octants of
    # 125 voxels (odd half-width: no voxel is equidistant from two seeds)
    comp = np.zeros((10, 10, 10), dtype=np.uint32)
    pts = [(x, y, z) for z in (2, 7) for y in (2, 7) for x in (2, 7)]
    sites = np.array([x + 10 * (y + 10 * z) for x, y, z in pts], dtype=np.uint32)
    cell = oracle.vt(comp, sites)
    z, y, x = np.indices((10, 10, 10))
    want = (x >= 5).astype(int) + 2 * (y >= 5) + 4 * (z >= 5)
    np.testing.assert_array_equal(cell, want.astype(np.uint32))
    assert np.all(np.bincount(cell.ravel()) == 125)


def test_vt_line_midpoint_tie_goes_to_lower_id():
    comp = np.zeros((1, 1, 7), dtype=np.uint32)
    cell = oracle.vt(comp, np.array([5, 1], dtype=np.uint32))   # ids: 0 at x=5, 1 at x=1
    # x = 3 is 2 hops from both sites and goes to id 0
    np.testing.assert_array_equal(cell.ravel(), [1, 1, 1, 0, 0, 0, 0])


def test_vt_single_seed_is_component_and_unseeded_is_none():
    rng = np.random.default_rng(7)
    band = brute.random_bands((8, 8, 8), 2, rng, smooth=True)
    cc = oracle.components(band, 2)
    # seed component 0 at its first voxel only
    cell = oracle.vt(cc.comp, np.array([cc.comp_first[0]], dtype=np.uint32))
    np.testing.assert_array_equal(cell == 0, cc.comp == 0)
    assert np.all(cell[cc.comp != 0] == NONE)


def test_vt_every_voxel_a_seed():
    rng = np.random.default_rng(8)
    band = brute.random_bands((3, 4, 5), 2, rng)
    comp = oracle.components(band, 2).comp
    sites = rng.permutation(comp.size).astype(np.uint32)
    cell = oracle.vt(comp, sites)
    want = np.empty(comp.size, dtype=np.uint32)
    want[sites] = np.arange(comp.size, dtype=np.uint32)
    np.testing.assert_array_equal(cell.ravel(), want)


def test_vt_respects_band_boundaries():
    # a wall of band 1 splits band 0 into two components; a site on the left
    # never claims the right side even though it is Euclidean-closer
    band = np.zeros((1, 5, 9), dtype=np.uint8)
    band[0, :, 4] = 1
    cc = oracle.components(band, 2)
    cell = oracle.vt(cc.comp, np.array([3, 8 + 9 * 4], dtype=np.uint32))
    assert np.all(cell[0, :, :4] == 0) and np.all(cell[0, :, 5:] == 1)
    assert np.all(cell[0, :, 4] == NONE)


# --------------------------------------------------------------------------
# site update (Sec. 3.1 centroid), exact rationals
@pytest.mark.parametrize("seed,weighted", [(0, False), (1, True), (2, True), (3, False), (4, True)])
def test_update_matches_fraction_bruteforce(seed, weighted):
    rng = np.random.default_rng(seed)
    band = brute.random_bands((5, 6, 7), 2, rng, smooth=True)
    comp = oracle.components(band, 2).comp
    sites = rng.choice(comp.size, size=9, replace=False).astype(np.uint32)
    cell = oracle.vt(comp, sites)
    w = rng.integers(0, 65536, size=comp.shape).astype(np.uint16) if weighted else None
    if weighted:
        w.ravel()[rng.integers(0, comp.size, size=20)] = 0
    got, ds = oracle.update(cell, sites, w)
    want = brute.update_fraction(cell, sites, w)
    np.testing.assert_array_equal(got, want)
    nx, ny = comp.shape[2], comp.shape[1]
    for s in range(len(sites)):
        a = np.array([sites[s] % nx, (sites[s] // nx) % ny, sites[s] // (nx * ny)], dtype=float)
        b = np.array([want[s] % nx, (want[s] // nx) % ny, want[s] // (nx * ny)], dtype=float)
        assert ds[s] == pytest.approx(np.linalg.norm(a - b), abs=0, rel=1e-15)


def test_update_box_centroid_and_half_integer_tie():
    # a 4x3x5 box (one cell): centroid (1.5, 1, 2); ties go down to x = 1
    cell = np.zeros((5, 3, 4), dtype=np.uint32)
    new, _ = oracle.update(cell, np.array([0], dtype=np.uint32))
    assert new[0] == 1 + 4 * (1 + 3 * 2)


def test_update_large_weights_exact():
    # near the top of the uint16 range the rational centroid is still exact
    cell = np.zeros((1, 1, 6), dtype=np.uint32)
    w = np.array([65535, 65535, 65535, 1, 65535, 65534], dtype=np.uint16).reshape(1, 1, 6)
    new, _ = oracle.update(cell, np.array([0], dtype=np.uint32), w)
    assert new[0] == brute.update_fraction(cell, [0], w)[0]


def test_update_zero_mass_keeps_site():
    cell = np.zeros((1, 2, 3), dtype=np.uint32)
    cell[0, 1, :] = NONE
    w = np.zeros((1, 2, 3), dtype=np.uint16)
    new, ds = oracle.update(cell, np.array([2, 5], dtype=np.uint32), w)
    assert list(new) == [2, 5] and list(ds) == [0.0, 0.0]


# --------------------------------------------------------------------------
# Algorithm 1 with fixed iterations
def _blobs_small(seed=3, shape=(20, 22, 24)):
    import synth
    f = synth.blobs_field(shape, seed)
    iso = synth.quantile_isovalues(f, [0.2, 0.4, 0.6, 0.8])
    band = oracle.bands(f, iso)
    cc = oracle.components(band, 5)
    return f, band, cc


def test_cvt_invariants_and_resume():
    import synth
    f, band, cc = _blobs_small()
    w = synth.gradient_weight(f)
    seeds = synth.seed_sites(cc.comp, cc.n_comp, w, 64.0, 11)
    T = 6
    r = oracle.cvt(cc.comp, seeds, w, T)
    # every voxel in exactly one cell (each component has a seed)
    assert not np.any(r.cell == NONE)
    # each cell lies in one component and is connected; its site is inside it
    site_comp = cc.comp.ravel()[seeds]
    np.testing.assert_array_equal(r.site_comp, site_comp)
    flat = r.cell.ravel()
    np.testing.assert_array_equal(cc.comp.ravel(), site_comp[flat])
    from scipy import ndimage
    struct = ndimage.generate_binary_structure(3, 1)
    for s in range(len(seeds)):
        mask = r.cell == s
        if mask.any():
            assert ndimage.label(mask, structure=struct)[1] == 1
            assert flat[r.sites[s]] == s
    # sum of cell counts per component equals the component size
    cnt = np.bincount(site_comp[flat].astype(np.int64), minlength=cc.n_comp)
    np.testing.assert_array_equal(cnt, cc.comp_size)
    # distinct sites stay distinct
    assert len(np.unique(r.sites)) == len(np.unique(seeds))
    # resume: T = T1 + T2
    r1 = oracle.cvt(cc.comp, seeds, w, 2)
    r2 = oracle.cvt(cc.comp, r1.sites, w, T - 2)
    np.testing.assert_array_equal(r2.cell, r.cell)
    np.testing.assert_array_equal(r2.sites, r.sites)
    np.testing.assert_allclose(np.concatenate([r1.mean_ds, r2.mean_ds]), r.mean_ds, rtol=0, atol=0)
    # T = 0 is the plain tessellation of the seeds
    r0 = oracle.cvt(cc.comp, seeds, w, 0)
    np.testing.assert_array_equal(r0.cell, oracle.vt(cc.comp, seeds))
    np.testing.assert_array_equal(r0.sites, seeds)


def test_cvt_steps_match_bruteforce_tiny():
    rng = np.random.default_rng(21)
    band = brute.random_bands((5, 5, 6), 2, rng, smooth=True)
    comp = oracle.components(band, 2).comp
    seeds = rng.choice(comp.size, size=6, replace=False).astype(np.uint32)
    w = rng.integers(1, 1000, size=comp.shape).astype(np.uint16)
    sites = seeds.copy()
    for _ in range(3):
        cell, _ = brute.vt_allpairs(comp, sites)
        sites = brute.update_fraction(cell, sites, w)
    cell, _ = brute.vt_allpairs(comp, sites)
    r = oracle.cvt(comp, seeds, w, 3)
    np.testing.assert_array_equal(r.sites, sites)
    np.testing.assert_array_equal(r.cell, cell)


def test_cvt_octants_fixed_point():
    comp = np.zeros((10, 10, 10), dtype=np.uint32)
    pts = [(x, y, z) for z in (2, 7) for y in (2, 7) for x in (2, 7)]
    sites = np.array([x + 10 * (y + 10 * z) for x, y, z in pts], dtype=np.uint32)
    r = oracle.cvt(comp, sites, None, 4)
    np.testing.assert_array_equal(r.sites, sites)
    assert np.all(r.mean_ds == 0.0)


def test_cvt_errors():
    comp = np.zeros((2, 2, 2), dtype=np.uint32)
    with pytest.raises(oracle.OracleError):
        oracle.cvt(comp, np.array([8], dtype=np.uint32), None, 1)
    with pytest.raises(oracle.OracleError):
        oracle.cvt(comp, np.array([0], dtype=np.uint32), None, -1)


# --------------------------------------------------------------------------
# statistics (Sec. 3.3 Aggregation)
@pytest.mark.parametrize("seed", range(3))
def test_stats_match_numpy(seed):
    rng = np.random.default_rng(seed)
    shape = (6, 7, 8)
    unit = rng.integers(0, 9, size=shape).astype(np.uint32)
    unit[0, 0, :3] = NONE
    m = 4
    x = rng.normal(loc=[[[[3.0]]], [[[-1.0]]], [[[0.0]]], [[[100.0]]]], scale=1.0, size=(m,) + shape).astype(np.float32)
    x[2, 1, 1, 1] = 1e30          # a value far above every edge
    x[2, 1, 1, 2] = -1e30
    edges = np.stack([np.linspace(-3, 3, 11) for _ in range(m)]).astype(np.float32)
    edges[3] = np.linspace(97, 103, 11)
    got = oracle.stats(unit, 10, x, edges, cov=True)     # unit 9 is empty
    n, mean, m2, vmin, vmax, hist, cv = brute.stats_numpy(unit, 10, x, edges, cov=True)
    np.testing.assert_array_equal(got.n, n)
    np.testing.assert_allclose(got.mean, mean, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(got.m2, m2, rtol=1e-10, atol=1e-10)
    np.testing.assert_array_equal(got.vmin, vmin)
    np.testing.assert_array_equal(got.vmax, vmax)
    np.testing.assert_array_equal(got.hist, hist)
    np.testing.assert_allclose(got.cov, cv, rtol=1e-10, atol=1e-8)
    assert got.n[9] == 0 and np.all(got.vmin[9] == np.inf) and np.all(got.vmax[9] == -np.inf)
    # population variance equals numpy's var (ddof = 0) unit by unit
    for u in range(9):
        sel = unit.ravel() == u
        assert got.var[u, 1] == pytest.approx(np.var(x[1].ravel()[sel].astype(np.float64)), rel=1e-12)


def test_stats_fraction_exact_tiny():
    from fractions import Fraction
    vals = np.array([[0.5, 0.25, 2.0, -1.0, 3.0]], dtype=np.float32)
    vals2 = np.array([[1.0, 2.0, 0.0, 4.0, 8.0]], dtype=np.float32)
    x = np.stack([vals, vals2]).reshape(2, 1, 1, 5)
    unit = np.zeros((1, 1, 5), dtype=np.uint32)
    got = oracle.stats(unit, 1, x, cov=True)
    a = [Fraction(float(v)) for v in vals.ravel()]
    b = [Fraction(float(v)) for v in vals2.ravel()]
    ma, mb = sum(a) / 5, sum(b) / 5
    assert got.mean[0, 0] == float(ma) and got.mean[0, 1] == float(mb)
    assert got.m2[0, 0] == pytest.approx(float(sum((v - ma) ** 2 for v in a)), rel=1e-15)
    assert got.cov[0, 1] == pytest.approx(float(sum((p - ma) * (q - mb) for p, q in zip(a, b))), rel=1e-15)
    assert got.cov[0, 0] == got.m2[0, 0] and got.cov[0, 2] == got.m2[0, 1]


def test_stats_histogram_edge_convention():
    # bin = number of interior edges <= x; below e_0 -> bin 0; >= e_B -> bin B-1
    edges = np.array([[0.0, 1.0, 2.0, 3.0]], dtype=np.float32)
    x = np.array([-5.0, 0.0, 0.999, 1.0, 2.5, 3.0, 9.0], dtype=np.float32).reshape(1, 1, 1, 7)
    unit = np.zeros((1, 1, 7), dtype=np.uint32)
    got = oracle.stats(unit, 1, x, edges)
    np.testing.assert_array_equal(got.hist[0, 0], [3, 1, 3])


def test_chan_merge_of_cells_equals_direct_components():
    import synth
    f, band, cc = _blobs_small(seed=5, shape=(16, 18, 20))
    seeds = synth.seed_sites(cc.comp, cc.n_comp, None, 40.0, 3)
    r = oracle.cvt(cc.comp, seeds, None, 2)
    rng = np.random.default_rng(0)
    x = np.stack([f, rng.normal(5.0, 2.0, size=f.shape).astype(np.float32)])
    S = len(seeds)
    cs = oracle.stats(r.cell, S, x, cov=True)
    comp_unit = np.where(r.cell == NONE, NONE, r.site_comp[np.minimum(r.cell, S - 1)])
    direct = oracle.stats(comp_unit, cc.n_comp, x, cov=True)
    acc = {}
    for s in range(S):
        c = int(r.site_comp[s])
        cur = acc.get(c, (0, np.zeros(2), np.zeros(2), np.zeros(3)))
        acc[c] = oracle.chan_merge(*cur, int(cs.n[s]), cs.mean[s], cs.m2[s], cs.cov[s])
    for c, (n, mean, m2, cv) in acc.items():
        assert n == direct.n[c]
        np.testing.assert_allclose(mean, direct.mean[c], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(m2, direct.m2[c], rtol=1e-10, atol=1e-9)
        np.testing.assert_allclose(cv, direct.cov[c], rtol=1e-10, atol=1e-9)


def test_mean_ds_decays_like_fig9():
    """Qualitative shape only (the paper's metric differs): the mean site move
    shrinks quickly over the first updates, as in the paper's Fig. 9."""
    import os
    import synth
    path = os.path.join(os.path.dirname(__file__), "golden", "fig9_mean_ds.txt")
    fig9 = np.loadtxt(path, comments="#")
    assert fig9.shape == (50, 4)
    paper_ratio = fig9[9, 1:] / fig9[0, 1:]          # update 10 vs update 1
    assert np.all(paper_ratio < 0.1)
    f = synth.fourier_field((40, 40, 40), 9, n_modes=64, kmax=6)
    iso = synth.quantile_isovalues(f, [0.25, 0.5, 0.75])
    cc = oracle.components(oracle.bands(f, iso), 4)
    w = synth.gradient_weight(f)
    seeds = synth.seed_sites(cc.comp, cc.n_comp, w, 256.0, 5)
    r = oracle.cvt(cc.comp, seeds, w, 10)
    assert r.mean_ds[0] > 0.5
    assert r.mean_ds[9] < 0.35 * r.mean_ds[0]


# ---------------------------------------------------------------------------
# Structured layout (Sec. 3.2.4, Fig. 5)

def test_layout_hand_example():
    """Worked by hand: sites 0 and 2 in component 0 (band 0), site 1 in
    component 1 (band 1); voxel 3 carries a label that is no site and voxel 6
    is unlabelled, so both are left out."""
    cell = np.array([1, 0, 0, 5, 1, 2, NONE, 2], dtype=np.uint32)
    L = oracle.layout(cell, [0, 1, 0], [0, 1], 2, 2)
    assert L.site_order.tolist() == [0, 2, 1]
    assert L.perm.tolist() == [1, 2, 5, 7, 0, 4]
    assert L.cell_off.tolist() == [0, 2, 4, 6]
    assert L.comp_off.tolist() == [0, 4, 6]
    assert L.band_off.tolist() == [0, 4, 6]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_layout_against_tuple_sort(seed):
    """Brute force: sort the placed voxels by the tuple (band, component,
    site, index) with Python's sort and count the ranges in plain loops."""
    rng = np.random.default_rng(seed)
    n, S, C, NB = 300, 17, 5, 4
    cell = rng.integers(0, S + 3, size=n).astype(np.uint32)
    cell[rng.random(n) < 0.1] = NONE
    site_comp = rng.integers(0, C + 1, size=S).astype(np.uint32)  # C = beyond the components
    comp_band = np.sort(rng.integers(0, NB, size=C)).astype(np.uint8)
    L = oracle.layout(cell, site_comp, comp_band, C, NB)

    def key(v):
        s = int(cell[v])
        c = min(int(site_comp[s]), C)
        b = int(comp_band[c]) if c < C else NB
        return (b, c, s, v)

    placed = [v for v in range(n) if cell[v] < S]
    assert L.perm.tolist() == sorted(placed, key=key)
    assert sorted(L.site_order.tolist(), key=lambda s: (min(int(site_comp[s]), C), s)) == L.site_order.tolist()
    assert sorted(L.site_order.tolist()) == list(range(S))
    for k in range(S):
        s = int(L.site_order[k])
        members = [v for v in L.perm[L.cell_off[k]:L.cell_off[k + 1]]]
        assert members == sorted(v for v in placed if cell[v] == s)
    for c in range(C):
        seg = L.perm[L.comp_off[c]:L.comp_off[c + 1]].tolist()
        assert seg == sorted((v for v in placed if site_comp[cell[v]] == c), key=key)
    for b in range(NB):
        seg = L.perm[L.band_off[b]:L.band_off[b + 1]].tolist()
        assert seg == sorted((v for v in placed if site_comp[cell[v]] < C and comp_band[site_comp[cell[v]]] == b),
                             key=key)


def test_extract_is_gather():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(3, 2, 3, 4)).astype(np.float32)
    perm = np.array([5, 0, 23, 7], dtype=np.uint32)
    out = oracle.extract(x, perm)
    for j in range(3):
        for k, v in enumerate(perm):
            z, r = divmod(int(v), 12)
            y, xx = divmod(r, 4)
            assert out[j, k] == x[j, z, y, xx]


# --------------------------------------------------------------------------
# stratified initial sites (Sec. 3.2.1, Eq. 3, Eq. 4)
from fractions import Fraction  # noqa: E402
import math  # noqa: E402

from oracle import seeding  # noqa: E402


def test_philox_known_answers():
    # known-answer vectors of Philox4x32-10 published with the generator
    # (Salmon et al., SC 2011, Random123 known-answer tests)
    cases = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
             ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
             ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
              (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for ctr, key, want in cases:
        assert oracle.philox4x32(ctr, key) == want


def _pieces(seed, shape=(20, 18, 22), n_bands=3):
    rng = np.random.default_rng(seed)
    band = brute.random_bands(shape, n_bands, rng, True)
    cc = oracle.components(band, n_bands)
    return rng, cc


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_seed_counts_closed_form_uniform(seed):
    # uniform mass: n_c = max(ceil(|C| / rho), 1) (Eq. 3 with m = 1)
    rng, cc = _pieces(seed)
    rho = int(rng.integers(20, 200))
    s = oracle.seed_stratified(cc.comp, cc.n_comp, None, None, rho=rho, block=8, seed=seed)
    got = np.bincount(cc.comp.ravel()[s], minlength=cc.n_comp)
    want = [max(math.ceil(int(n) / rho), 1) for n in cc.comp_size]
    np.testing.assert_array_equal(got, want)


def test_seed_counts_weighted_fraction():
    rng, cc = _pieces(5)
    w = rng.integers(0, 1000, size=cc.comp.shape).astype(np.uint16)
    rho = 37
    s = oracle.seed_stratified(cc.comp, cc.n_comp, w, None, rho=rho, block=8, seed=3)
    got = np.bincount(cc.comp.ravel()[s], minlength=cc.n_comp)
    m = w.ravel().astype(np.int64)
    total = int(m.sum())
    n = m.size
    for c in range(cc.n_comp):
        mc = int(m[cc.comp.ravel() == c].sum())
        want = max(math.ceil(Fraction(mc * n, rho * total)), 1)
        assert got[c] == want, c


def test_apportion_is_largest_remainder():
    # Hamilton's method: every share is floor or ceil of the quota, the total is
    # n_c, and no block that was rounded down has a larger remainder (or an
    # equal remainder and a lower block index) than one that was rounded up
    rng = np.random.default_rng(11)
    for _ in range(300):
        k = int(rng.integers(1, 12))
        masses = [int(v) for v in rng.integers(0, 50, size=k)]
        if sum(masses) == 0:
            masses[0] = 1
        blocks = sorted(int(b) for b in rng.choice(1000, size=k, replace=False))
        n_c = int(rng.integers(1, 40))
        got = seeding.apportion(n_c, masses, blocks)
        total = sum(masses)
        q = [Fraction(n_c * m, total) for m in masses]
        assert sum(got) == n_c
        up = [i for i in range(k) if got[i] == math.floor(q[i]) + 1]
        down = [i for i in range(k) if got[i] == math.floor(q[i])]
        assert len(up) + len(down) == k
        for i in up:
            for j in down:
                fi, fj = q[i] - math.floor(q[i]), q[j] - math.floor(q[j])
                assert fi > fj or (fi == fj and blocks[i] < blocks[j])


def test_seed_placement_bruteforce_tiny():
    # site j of a pair holds point p_j = floor((o + j m(b)) / n_b) in its
    # cumulative-mass interval, walking the pair's voxels in linear order
    rng, cc = _pieces(7, shape=(9, 10, 11), n_bands=2)
    w = rng.integers(0, 9, size=cc.comp.shape).astype(np.uint16)
    block, rho, key = 4, 6, 0x1234_5678_9ABC
    s = oracle.seed_stratified(cc.comp, cc.n_comp, w, None, rho=rho, block=block, seed=key)
    nz, ny, nx = cc.comp.shape
    comp = cc.comp.ravel()
    m = w.ravel().astype(np.int64)
    blk = seeding.block_index(cc.comp.shape, block)
    k = 0
    for c in range(cc.n_comp):
        mine = s[comp[s] == c]
        if m[comp == c].sum() == 0:
            assert list(mine) == [int(np.flatnonzero(comp == c)[0])]
            k += 1
            continue
        for b in sorted(set(blk[mine].tolist())):
            vox = [v for v in range(comp.size) if comp[v] == c and blk[v] == b]
            mb = int(sum(m[v] for v in vox))
            got = [int(v) for v in mine if blk[v] == b]
            nb = len(got)
            o = seeding.pair_offset(key, b, c, mb)
            for j in range(nb):
                p = (o + j * mb) // nb
                acc = 0
                for v in vox:
                    if acc <= p < acc + m[v]:
                        assert got[j] == v
                        break
                    acc += m[v]
                else:
                    raise AssertionError("point beyond the pair's mass")
            k += nb
    assert k == len(s)


def test_seed_uniform_pair_spacing_order_and_determinism():
    rng, cc = _pieces(9, shape=(24, 24, 24), n_bands=2)
    s = oracle.seed_stratified(cc.comp, cc.n_comp, None, None, rho=50, block=8, seed=99)
    comp = cc.comp.ravel()
    blk = seeding.block_index(cc.comp.shape, 8)
    key = comp[s].astype(np.int64) * (blk.max() + 1) + blk[s]
    assert np.all(np.diff(key) >= 0)  # numbered by (component, block)
    # uniform mass: the picks of a pair are distinct and evenly spaced in the pair's order
    for c, b in set(zip(comp[s].tolist(), blk[s].tolist())):
        vox = np.flatnonzero((comp == c) & (blk == b))
        picks = np.searchsorted(vox, s[(comp[s] == c) & (blk[s] == b)])
        nb, kb = len(picks), len(vox)
        d = np.diff(picks)
        assert len(set(picks.tolist())) == nb
        assert np.all((d == kb // nb) | (d == -(-kb // nb)))
    np.testing.assert_array_equal(s, oracle.seed_stratified(cc.comp, cc.n_comp, None, None, rho=50, block=8,
                                                            seed=99))
    assert not np.array_equal(s, oracle.seed_stratified(cc.comp, cc.n_comp, None, None, rho=50, block=8, seed=98))


def test_seed_lut_and_zero_mass():
    rng, cc = _pieces(12)
    w = rng.integers(0, 300, size=cc.comp.shape).astype(np.uint16)
    ones = np.ones(65536, dtype=np.uint32)
    np.testing.assert_array_equal(oracle.seed_stratified(cc.comp, cc.n_comp, w, ones, rho=40, block=8, seed=1),
                                  oracle.seed_stratified(cc.comp, cc.n_comp, None, None, rho=40, block=8, seed=1))
    # a table that zeroes every weight below 150: no site on a zero-mass voxel
    lut = np.arange(65536, dtype=np.uint32)
    lut[:150] = 0
    s = oracle.seed_stratified(cc.comp, cc.n_comp, w, lut, rho=40, block=8, seed=1)
    comp = cc.comp.ravel()
    m = lut[w.ravel()]
    for v in s:
        c = comp[v]
        if m[comp == c].sum() > 0:
            assert m[v] > 0
        else:
            assert v == np.flatnonzero(comp == c)[0]


def test_seed_block_index_from_linear_index():
    # block of voxel v from its linear index v = x + nx (y + ny z)
    shape, B = (13, 7, 10), 4
    nz, ny, nx = shape
    got = seeding.block_index(shape, B)
    nbx, nby = -(-nx // B), -(-ny // B)
    for v in range(nx * ny * nz):
        x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
        assert got[v] == x // B + nbx * (y // B + nby * (z // B))


# --------------------------------------------------------------------------
# joint moments up to fourth order (Sec. 4.4: covariance, coskewness, cokurtosis)
from scipy import stats as sstats  # noqa: E402


def test_comoments_diagonal_match_scipy_moment():
    rng = np.random.default_rng(21)
    unit = rng.integers(0, 5, size=(6, 7, 8)).astype(np.uint32)
    unit.ravel()[::11] = oracle.NONE_ID
    x = rng.gamma(2.0, size=(3, 6, 7, 8)).astype(np.float32)
    mo = oracle.comoments(unit, 6, x)
    t2, t3, t4 = (oracle.tuples(3, r) for r in (2, 3, 4))
    for u in range(5):
        sel = unit.ravel() == u
        n = int(sel.sum())
        assert mo.n[u] == n
        for j in range(3):
            v = x[j].ravel()[sel].astype(np.float64)
            np.testing.assert_allclose(mo.m2[u, t2.index((j, j))], n * sstats.moment(v, 2), rtol=1e-12)
            np.testing.assert_allclose(mo.m3[u, t3.index((j, j, j))], n * sstats.moment(v, 3), rtol=1e-9,
                                       atol=1e-9 * n * v.std() ** 3)
            np.testing.assert_allclose(mo.m4[u, t4.index((j, j, j, j))], n * sstats.moment(v, 4), rtol=1e-12)
    assert mo.n[5] == 0 and np.all(mo.m4[5] == 0) and np.all(mo.mean[5] == 0)


def test_comoments_exact_cross_terms_fraction():
    # small integers: every cross moment checked in exact rational arithmetic
    rng = np.random.default_rng(22)
    unit = rng.integers(0, 3, size=(3, 4, 5)).astype(np.uint32)
    x = rng.integers(-4, 5, size=(3, 3, 4, 5)).astype(np.float32)
    mo = oracle.comoments(unit, 3, x)
    for u in range(3):
        sel = unit.ravel() == u
        rows = [[Fraction(int(v)) for v in x[j].ravel()[sel]] for j in range(3)]
        n = len(rows[0])
        mu = [sum(r) / n for r in rows]
        d = [[v - mu[j] for v in rows[j]] for j in range(3)]
        for r, got in ((2, mo.m2[u]), (3, mo.m3[u]), (4, mo.m4[u])):
            for k, tup in enumerate(oracle.tuples(3, r)):
                want = sum(math.prod(d[i][p] for i in tup) for p in range(n))
                assert got[k] == pytest.approx(float(want), rel=1e-12, abs=1e-9)


def test_comoments_symmetric_and_shift_invariant():
    # mirrored data (x and 2c - x in equal numbers) has zero odd central moments;
    # central moments do not change when a constant is added
    rng = np.random.default_rng(23)
    half = (np.round(rng.normal(size=(2, 500)) * 1024) / 1024).astype(np.float32)  # multiples of 2^-10
    x = np.concatenate([half, 2 * 3.0 - half], axis=1).astype(np.float32)
    unit = np.zeros(x.shape[1], dtype=np.uint32)
    mo = oracle.comoments(unit, 1, x)
    scale = mo.m2[0, 0] ** 1.5
    assert np.all(np.abs(mo.m3[0]) <= 1e-9 * scale)
    # shift by 8 (exact in float32 for multiples of 2^-10 this small): central moments are unchanged
    sh = (x + np.float32(8.0)).astype(np.float32)
    mo2 = oracle.comoments(unit, 1, sh)
    np.testing.assert_allclose(mo2.mean, mo.mean + 8.0, rtol=1e-12)
    np.testing.assert_allclose(mo2.m4, mo.m4, rtol=1e-12)
    np.testing.assert_allclose(mo2.m3, mo.m3, rtol=0, atol=1e-9 * scale)
