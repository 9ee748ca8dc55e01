"""GPU parity of the labelling rows against the CPU oracle (bit-exact).

Isobands (Sec. 3.1), components (Sec. 3.1), the restricted Voronoi pass
(Eq. 1), the snapped centroid update (Sec. 3.1) and the Lloyd loop
(Algorithm 1) are integer computations, so the GPU library must reproduce the
oracle's labels, tables and sites exactly.  Every call goes through the C ABI
(``paper_2208_06970_amd`` is a ctypes marshalling layer).
"""
import numpy as np
import pytest

import oracle
import paper_2208_06970_amd as L
import synth
from tests import brute
from tests.gpu_util import banner, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(params=[L.VT_LEVELS, L.VT_BRICKS], ids=["levels", "bricks"])
def engine(request):
    """Run a Voronoi test with each schedule of the passes (same regions)."""
    prev = L.lsrvt_set_vt_engine(request.param)
    yield request.param
    L.lsrvt_set_vt_engine(prev)
NONE = oracle.NONE_ID


def _field(shape, seed, kind="fourier"):
    if kind == "blobs":
        return synth.blobs_field(shape, seed)
    return synth.fourier_field(shape, seed, n_modes=128, kmax=max(2.0, min(shape) / 4))


def _labels(f, iso):
    banner(f"isobands+components shape={f.shape} K={len(iso)}")
    band_d, st = L.lsrvt_isobands(dev(f), iso)
    cc = L.lsrvt_components(band_d, len(iso) + 1)
    return band_d, st, cc


# --------------------------------------------------------------------------
# isobands
@pytest.mark.parametrize("shape,K,seed", [((64, 64, 64), 4, 1), ((37, 29, 45), 8, 2), ((1, 1, 1000), 3, 3),
                                          ((5, 7, 9), 0, 4), ((20, 30, 17), 40, 5), ((33, 1, 31), 254, 6)])
def test_isobands_parity(shape, K, seed):
    f = _field(shape, seed)
    rng = np.random.default_rng(seed)
    f.ravel()[rng.integers(0, f.size, 7)] = np.inf
    f.ravel()[rng.integers(0, f.size, 7)] = -np.inf
    iso = synth.quantile_isovalues(f[np.isfinite(f)], np.linspace(0, 1, K + 2)[1:-1]) if K else np.zeros(0, np.float32)
    if K:
        f.ravel()[:K] = iso          # values equal to an isovalue join the lower band
    banner(f"isobands shape={shape} K={K}")
    band, st = L.lsrvt_isobands(dev(f), iso)
    np.testing.assert_array_equal(host(band), oracle.bands(f, iso))
    assert int(host(st)[0]) == 0


def test_isobands_nan_flag_and_errors():
    f = np.zeros((3, 4, 21), dtype=np.float32)
    f[1, 2, 17] = np.nan
    banner("isobands NaN flag")
    _, st = L.lsrvt_isobands(dev(f), np.array([0.5], np.float32))
    assert int(host(st)[0]) & 1
    with pytest.raises(L.LsrvtError) as e:
        L.lsrvt_isobands(dev(f), np.array([1.0, 1.0], np.float32))
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LsrvtError) as e:
        L.lsrvt_isobands(dev(f), np.array([np.inf], np.float32))
    assert e.value.code == L.EINVAL


# --------------------------------------------------------------------------
# components
def _check_components(cc, want):
    assert cc.n_comp == want.n_comp
    np.testing.assert_array_equal(host(cc.comp, np.uint32), want.comp)
    np.testing.assert_array_equal(host(cc.comp_band), want.comp_band)
    np.testing.assert_array_equal(host(cc.comp_size).astype(np.uint64), want.comp_size)
    np.testing.assert_array_equal(host(cc.comp_first, np.uint32), want.comp_first)
    np.testing.assert_array_equal(host(cc.band_offset, np.uint32), want.band_offset)


@pytest.mark.parametrize("shape,K,seed,kind", [((64, 64, 64), 4, 1, "blobs"), ((37, 29, 45), 6, 2, "fourier"),
                                               ((70, 33, 18), 3, 3, "fourier"), ((1, 1, 777), 2, 4, "fourier"),
                                               ((1, 41, 67), 5, 5, "fourier"), ((1, 1, 1), 0, 6, "fourier"),
                                               ((9, 130, 3), 7, 7, "fourier")])
def test_components_parity(shape, K, seed, kind):
    f = _field(shape, seed, kind)
    iso = synth.quantile_isovalues(f, np.linspace(0, 1, K + 2)[1:-1]) if K else np.zeros(0, np.float32)
    band_d, _, cc = _labels(f, iso)
    want = oracle.components(oracle.bands(f, iso), K + 1)
    _check_components(cc, want)


def test_components_checkerboard_and_capacity_retry():
    z, y, x = np.indices((19, 23, 35))
    band = ((x + y + z) % 2).astype(np.uint8)      # every voxel its own component
    banner("components checkerboard")
    cc = L.lsrvt_components(dev(band), 2, cap_comp=16)     # forces ECAPACITY then a retry
    _check_components(cc, oracle.components(band, 2))


def test_components_random_noise_bands():
    rng = np.random.default_rng(11)
    band = brute.random_bands((40, 36, 50), 3, rng)
    banner("components noise")
    cc = L.lsrvt_components(dev(band), 3)
    _check_components(cc, oracle.components(band, 3))


# --------------------------------------------------------------------------
# Voronoi pass and update
@pytest.mark.parametrize("shape,K,seed,S", [((64, 64, 64), 4, 1, 600), ((37, 29, 45), 6, 2, 300),
                                            ((1, 1, 500), 2, 3, 9), ((1, 50, 70), 3, 4, 40),
                                            ((50, 40, 33), 1, 5, 1), ((17, 16, 48), 5, 6, 2000)])
def test_vt_parity(shape, K, seed, S, engine):
    f = _field(shape, seed, "blobs" if shape == (64, 64, 64) else "fourier")
    iso = synth.quantile_isovalues(f, np.linspace(0, 1, K + 2)[1:-1])
    band_d, _, cc = _labels(f, iso)
    rng = np.random.default_rng(seed)
    sites = rng.integers(0, f.size, size=S).astype(np.uint32)
    sites[-1] = sites[0]                            # duplicate: higher id keeps an empty cell
    banner(f"vt shape={shape} S={S}")
    cell = L.lsrvt_vt(band_d, dev(sites))
    want = oracle.vt(host(cc.comp, np.uint32), sites)
    np.testing.assert_array_equal(host(cell, np.uint32), want)
    if S > 1:
        assert not np.any(host(cell, np.uint32) == S - 1)


def test_vt_every_voxel_a_site(engine):
    rng = np.random.default_rng(3)
    band = brute.random_bands((6, 17, 19), 2, rng, smooth=True)
    comp = oracle.components(band, 2).comp
    sites = rng.permutation(band.size).astype(np.uint32)
    banner("vt every voxel a site")
    cell = L.lsrvt_vt(dev(band), dev(sites))
    np.testing.assert_array_equal(host(cell, np.uint32), oracle.vt(comp, sites))


def test_vt_octants_and_errors(engine):
    band = np.zeros((10, 10, 10), dtype=np.uint8)
    pts = [(x, y, z) for z in (2, 7) for y in (2, 7) for x in (2, 7)]
    sites = np.array([x + 10 * (y + 10 * z) for x, y, z in pts], dtype=np.uint32)
    banner("vt octants")
    cell = host(L.lsrvt_vt(dev(band), dev(sites)), np.uint32)
    z, y, x = np.indices((10, 10, 10))
    np.testing.assert_array_equal(cell, ((x >= 5) + 2 * (y >= 5) + 4 * (z >= 5)).astype(np.uint32))
    with pytest.raises(L.LsrvtError) as e:
        L.lsrvt_vt(dev(band), dev(np.array([5, 1000], dtype=np.uint32)))
    assert e.value.code == L.EINVAL


@pytest.mark.parametrize("weighted,seed", [(False, 1), (True, 2), (True, 3)])
def test_update_parity(weighted, seed):
    shape = (30, 41, 37)
    f = _field(shape, seed)
    iso = synth.quantile_isovalues(f, [0.3, 0.6])
    band = oracle.bands(f, iso)
    comp = oracle.components(band, 3).comp
    rng = np.random.default_rng(seed)
    sites = rng.choice(f.size, size=150, replace=False).astype(np.uint32)
    cell = oracle.vt(comp, sites)
    w = None
    if weighted:
        w = rng.integers(0, 65536, size=shape).astype(np.uint16)
        w[rng.random(shape) < 0.1] = 0
        w[cell == cell.ravel()[0]] = 0               # a whole cell with zero mass keeps its site
    want, want_ds = oracle.update(cell, sites, w)
    banner(f"update weighted={weighted}")
    s_d = dev(sites)
    _, ds = L.lsrvt_update(dev(cell), s_d, None if w is None else dev(w))
    np.testing.assert_array_equal(host(s_d, np.uint32), want)
    np.testing.assert_allclose(host(ds), want_ds, rtol=1e-15, atol=0)


# --------------------------------------------------------------------------
# Lloyd loop
def _cvt_case(f, iso, weights, rho, seed, T):
    band_d, _, cc = _labels(f, iso)
    comp = host(cc.comp, np.uint32)
    want_cc = oracle.components(oracle.bands(f, iso), len(iso) + 1)
    np.testing.assert_array_equal(comp, want_cc.comp)
    seeds = synth.seed_sites(want_cc.comp, want_cc.n_comp, weights, rho, seed)
    want = oracle.cvt(want_cc.comp, seeds, weights, T)
    banner(f"cvt shape={f.shape} S={len(seeds)} T={T}")
    got = L.lsrvt_cvt(band_d, cc.comp, dev(seeds), None if weights is None else dev(weights), T)
    np.testing.assert_array_equal(host(got.site_comp, np.uint32), want.site_comp)
    np.testing.assert_array_equal(host(got.sites, np.uint32), want.sites)
    np.testing.assert_array_equal(host(got.cell, np.uint32), want.cell)
    np.testing.assert_allclose(got.mean_ds, want.mean_ds, rtol=1e-12, atol=1e-15)
    return got


def test_cvt_blobs_64(engine):
    wl = synth.blobs_workload()
    _cvt_case(wl.field, wl.iso, None, wl.rho, 5, wl.iters)


@pytest.mark.parametrize("shape,T,seed", [((37, 29, 45), 6, 2), ((48, 20, 33), 0, 3), ((1, 64, 90), 5, 4)])
def test_cvt_weighted_ragged(shape, T, seed, engine):
    f = _field(shape, seed)
    iso = synth.quantile_isovalues(f, [0.25, 0.5, 0.75])
    _cvt_case(f, iso, synth.gradient_weight(f), 96.0, seed, T)


def test_cvt_errors_and_determinism(engine):
    f = _field((20, 21, 22), 9)
    iso = synth.quantile_isovalues(f, [0.5])
    band_d, _, cc = _labels(f, iso)
    seeds = np.array([3, 100, 2000], dtype=np.uint32)
    with pytest.raises(L.LsrvtError) as e:
        L.lsrvt_cvt(band_d, cc.comp, dev(np.array([3, f.size], dtype=np.uint32)), None, 2)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.LsrvtError) as e:
        L.lsrvt_cvt(band_d, cc.comp, dev(seeds), None, -1)
    assert e.value.code == L.EINVAL
    a = L.lsrvt_cvt(band_d, cc.comp, dev(seeds), None, 4)
    b = L.lsrvt_cvt(band_d, cc.comp, dev(seeds), None, 4)
    assert np.array_equal(host(a.cell), host(b.cell)) and np.array_equal(host(a.sites), host(b.sites))


@pytest.mark.parametrize("grid", [256, 1024, 16384])
def test_cvt_every_relaxation_grid(grid):
    """Each relaxation-round grid the autotuner may choose gives the oracle's
    Lloyd loop bit for bit (the rounds' workgroups only walk the bricks with
    another stride)."""
    prev_e = L.lsrvt_set_vt_engine(L.VT_BRICKS)
    prev = L.lsrvt_set_tuning(L.TUNE_BR_GRID, grid)
    try:
        f = _field((40, 36, 90), 11)
        iso = synth.quantile_isovalues(f, [0.3, 0.6])
        _cvt_case(f, iso, synth.gradient_weight(f), 300.0, 11, 4)
    finally:
        L.lsrvt_set_tuning(L.TUNE_BR_GRID, prev)
        L.lsrvt_set_vt_engine(prev_e)


@pytest.mark.parametrize("bits", [0, 64, 20, 30])
def test_cvt_every_key_width(bits):
    """Narrow keys (the default here), wide keys, and narrow keys with so
    wide an id field that distances outgrow the rest (30 id bits leave
    distances below 2: every pass of this volume outgrows them and is
    repeated with wide keys) all give the oracle's Lloyd loop bit for bit."""
    prev_e = L.lsrvt_set_vt_engine(L.VT_BRICKS)
    prev = L.lsrvt_set_tuning(L.TUNE_KEY_BITS, bits)
    try:
        f = _field((40, 36, 90), 12)
        iso = synth.quantile_isovalues(f, [0.3, 0.6])
        _cvt_case(f, iso, synth.gradient_weight(f), 300.0, 12, 4)
    finally:
        L.lsrvt_set_tuning(L.TUNE_KEY_BITS, prev)
        L.lsrvt_set_vt_engine(prev_e)


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("bits", [0, 64])
def test_cvt_every_reset_mode(mode, bits):
    """Incremental relaxation passes that reset the moved sites' voxels by
    their own kernel, or in the first round as it reads them, with narrow
    and wide keys: the oracle's Lloyd loop bit for bit.  Two volumes: a
    weighted one with three isovalues (about 200 voxels per site) and an
    unweighted one with one isovalue and wider cells (about 900)."""
    prev_e = L.lsrvt_set_vt_engine(L.VT_BRICKS)
    prev = L.lsrvt_set_tuning(L.TUNE_RESET, mode)
    prev_b = L.lsrvt_set_tuning(L.TUNE_KEY_BITS, bits)
    try:
        f = _field((48, 40, 70), 13)
        iso = synth.quantile_isovalues(f, [0.25, 0.5, 0.75])
        _cvt_case(f, iso, synth.gradient_weight(f), 200.0, 13, 5)
        f = _field((33, 47, 29), 14)
        iso = synth.quantile_isovalues(f, [0.5])
        _cvt_case(f, iso, None, 900.0, 14, 4)
    finally:
        L.lsrvt_set_tuning(L.TUNE_KEY_BITS, prev_b)
        L.lsrvt_set_tuning(L.TUNE_RESET, prev)
        L.lsrvt_set_vt_engine(prev_e)


def test_update_and_loop_with_every_voxel_a_site():
    """More distinct cells than the LDS tables of the centroid sums hold
    (512 per 64x8x8 tile in lsrvt_update, 256 per 16^3 brick in the sums a
    Voronoi pass takes for the update that follows): every voxel a site, so
    the global-atomic fallbacks run; bit-exact against the oracle."""
    shape = (16, 24, 80)
    rng = np.random.default_rng(21)
    band = brute.random_bands(shape, 2, rng, smooth=True)
    comp = oracle.components(band, 2).comp
    sites = rng.permutation(band.size).astype(np.uint32)
    w = rng.integers(0, 65536, size=shape).astype(np.uint16)
    banner("update and loop, every voxel a site")
    cell = oracle.vt(comp, sites)
    want, want_ds = oracle.update(cell, sites, w)
    s_d = dev(sites)
    _, ds = L.lsrvt_update(dev(cell), s_d, dev(w))
    np.testing.assert_array_equal(host(s_d, np.uint32), want)
    np.testing.assert_allclose(host(ds), want_ds, rtol=1e-15, atol=0)
    for eng in (L.VT_LEVELS, L.VT_BRICKS):
        prev = L.lsrvt_set_vt_engine(eng)
        try:
            b = dev(band)
            g = L.lsrvt_components(b, 2)
            r = L.lsrvt_cvt(b, g.comp, dev(sites), dev(w), 2)
        finally:
            L.lsrvt_set_vt_engine(prev)
        ref = oracle.cvt(comp, sites, w, 2)
        np.testing.assert_array_equal(host(r.sites, np.uint32), ref.sites)
        np.testing.assert_array_equal(host(r.cell, np.uint32), ref.cell)
