"""GPU parity of the structured hierarchical layout (Sec. 3.2.4 "Data
Reduction and Structured Data Layout", Fig. 5) and of the raw-data
extraction against the oracle.  Everything here is integer or a copy, so
every comparison is bit-exact.
"""
import numpy as np
import pytest

import oracle
import paper_2208_06970_amd as L
import synth
from tests.gpu_util import banner, dev, host

pytestmark = pytest.mark.gpu
NONE = oracle.NONE_ID


def _check(cell, site_comp, comp_band, n_comp, n_bands, shape):
    cell = np.ascontiguousarray(cell, dtype=np.uint32).reshape(shape)
    want = oracle.layout(cell, site_comp, comp_band, n_comp, n_bands)
    got = L.lsrvt_layout(dev(cell), dev(np.asarray(site_comp, dtype=np.uint32)),
                         dev(np.asarray(comp_band, dtype=np.uint8)), n_comp, n_bands)
    assert got.n_placed == len(want.perm)
    np.testing.assert_array_equal(host(got.perm, np.uint32), want.perm)
    np.testing.assert_array_equal(host(got.site_order, np.uint32), want.site_order)
    np.testing.assert_array_equal(host(got.cell_off, np.uint32), want.cell_off)
    np.testing.assert_array_equal(host(got.comp_off, np.uint32), want.comp_off)
    np.testing.assert_array_equal(host(got.band_off, np.uint32), want.band_off)
    return got, want


def test_layout_pipeline_fourier():
    shape = (40, 48, 56)
    banner(f"layout fourier {shape}")
    wl = synth.fourier_workload(shape=shape, seed=11, n_iso=6, iters=2, rho=96.0)
    band = oracle.bands(wl.field, wl.iso)
    cc = oracle.components(band, wl.n_bands)
    seeds = synth.workload_sites(wl, cc.comp, cc.n_comp)
    r = oracle.cvt(cc.comp, seeds, wl.weights, 2)
    site_comp = cc.comp.ravel()[r.sites]
    got, want = _check(r.cell, site_comp, cc.comp_band, cc.n_comp, wl.n_bands, shape)
    # extraction in layout order
    x = np.ascontiguousarray(wl.variables[:3])
    out = L.lsrvt_extract(dev(x), got.perm)
    np.testing.assert_array_equal(host(out), oracle.extract(x, want.perm))


def test_layout_many_cells_per_tile_ragged():
    # random labels: far more distinct cells per 4096-voxel tile than the
    # small and medium tables hold, so every tile takes the whole-tile path
    rng = np.random.default_rng(5)
    shape = (3, 37, 113)  # 12543 voxels: three full tiles and a ragged one
    n = int(np.prod(shape))
    S = 5000
    cell = rng.integers(0, S, size=n).astype(np.uint32)
    cell[rng.random(n) < 0.05] = NONE
    cell[rng.random(n) < 0.01] = S + 7  # not a site id: left out
    n_comp = 40
    site_comp = rng.integers(0, n_comp + 3, size=S).astype(np.uint32)  # some beyond n_comp
    comp_band = np.sort(rng.integers(0, 5, size=n_comp)).astype(np.uint8)
    banner(f"layout random labels {shape} S={S}")
    _check(cell, site_comp, comp_band, n_comp, 6, shape)


def test_layout_mixed_tiles():
    # half the volume has large cells (common path), the rest one cell per voxel
    rng = np.random.default_rng(9)
    shape = (8, 32, 64)
    n = int(np.prod(shape))
    S = 3000
    cell = np.repeat(np.arange(n // 512, dtype=np.uint32), 512)[:n]
    cell[n // 2:] = rng.integers(0, S, size=n - n // 2)
    site_comp = np.sort(rng.integers(0, 10, size=S)).astype(np.uint32)
    comp_band = np.array([0, 0, 1, 1, 1, 2, 3, 3, 3, 3], dtype=np.uint8)
    banner(f"layout mixed tiles {shape}")
    _check(cell, site_comp, comp_band, 10, 4, shape)


def test_layout_every_table_size():
    """Tiles of 4096 voxels with 1, 256, 257, 400, 640, 641, 2000 and 4096
    distinct cells: the small table (up to 256), the medium one (up to 640)
    and the whole-tile one, at and across both limits; cells shared between
    tiles, voxels of a tile in random order for half of them."""
    rng = np.random.default_rng(17)
    shape = (8, 64, 64)  # one tile per z-plane
    S = 5000
    parts = []
    for k, d in enumerate([1, 256, 257, 400, 640, 641, 2000, 4096]):
        local = (np.arange(4096) * d) // 4096
        if k % 2:
            local = rng.permutation(local)
        parts.append(((local + 613 * k) % S).astype(np.uint32))
    cell = np.concatenate(parts)
    cell[rng.random(cell.size) < 0.02] = NONE
    site_comp = np.sort(rng.integers(0, 12, size=S)).astype(np.uint32)
    comp_band = np.sort(rng.integers(0, 4, size=12)).astype(np.uint8)
    banner(f"layout every table size {shape}")
    _check(cell, site_comp, comp_band, 12, 4, shape)


def test_layout_edge_cases():
    shape = (1, 1, 4097)
    banner("layout edges: no sites, one site, all NONE")
    cell = np.full(shape, NONE, dtype=np.uint32)
    got, _ = _check(cell, np.zeros(0, np.uint32), np.zeros(1, np.uint8), 1, 1, shape)
    assert got.n_placed == 0
    cell = np.zeros(shape, dtype=np.uint32)
    _check(cell, np.zeros(1, np.uint32), np.zeros(1, np.uint8), 1, 1, shape)
    cell[0, 0, ::3] = NONE
    _check(cell, np.zeros(1, np.uint32), np.zeros(1, np.uint8), 1, 3, shape)


def test_layout_deterministic_and_reusable_workspace():
    rng = np.random.default_rng(3)
    shape = (16, 64, 64)
    cell = rng.integers(0, 700, size=shape).astype(np.uint32)
    site_comp = rng.integers(0, 8, size=700).astype(np.uint32)
    comp_band = np.sort(rng.integers(0, 3, size=8)).astype(np.uint8)
    banner("layout determinism")
    ws = L.Workspace()
    a = L.lsrvt_layout(dev(cell), dev(site_comp), dev(comp_band), 8, 3, ws=ws)
    b = L.lsrvt_layout(dev(cell), dev(site_comp), dev(comp_band), 8, 3, ws=ws)
    for k in ("perm", "site_order", "cell_off", "comp_off", "band_off"):
        assert np.array_equal(host(getattr(a, k)), host(getattr(b, k))), k


def test_layout_host_validation():
    banner("layout host validation")
    cell = dev(np.zeros((2, 2, 2), np.uint32))
    sc = dev(np.zeros(1, np.uint32))
    cb = dev(np.zeros(1, np.uint8))
    with pytest.raises(L.LsrvtError):
        L.lsrvt_layout(cell, sc, cb, 1, 0)
    with pytest.raises(L.LsrvtError):
        L.lsrvt_layout(cell, sc, cb, 1, 256)
