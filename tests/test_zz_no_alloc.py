"""lsrvt_update_noalloc (the site update with the library's fixed per-GPU
scratch, for callers that cannot allocate) against lsrvt_update (caller
workspace) on the same inputs, bit for bit: two calls in a row, the second
on a smaller input, so stale scratch contents of the first call would show.
Sizes beyond the scratch limit are refused before any launch."""
import numpy as np
import pytest

import oracle
import paper_2208_06970_amd as L
import synth
from tests.gpu_util import banner, dev, host

pytestmark = pytest.mark.gpu


def _case(shape, seed, rho, weighted):
    f = synth.fourier_field(shape, seed, n_modes=64, kmax=8)
    iso = synth.quantile_isovalues(f, [0.25, 0.5, 0.75])
    band = oracle.bands(f, iso)
    cc = oracle.components(band, 4)
    w = synth.gradient_weight(f) if weighted else None
    seeds = synth.seed_sites(cc.comp, cc.n_comp, w, rho, seed + 1)
    cell = oracle.vt(cc.comp, seeds)
    return cell, seeds, w


def test_update_noalloc_matches_update_twice():
    cases = [((48, 40, 56), 31, 64.0, True), ((20, 24, 18), 32, 16.0, False)]
    for shape, seed, rho, weighted in cases:
        cell, seeds, w = _case(shape, seed, rho, weighted)
        banner(f"update_noalloc: shape={shape} sites={len(seeds)} weighted={weighted}")
        d_cell = dev(cell)
        d_w = None if w is None else dev(w)
        s_ref, ds_ref = L.lsrvt_update(d_cell, dev(seeds), d_w)
        s_na, ds_na = L.lsrvt_update_noalloc(d_cell, dev(seeds), d_w)
        np.testing.assert_array_equal(host(s_na), host(s_ref))
        np.testing.assert_array_equal(host(ds_na), host(ds_ref))
        want, want_ds = oracle.update(cell, seeds, w)
        np.testing.assert_array_equal(host(s_na, np.uint32), want)


def test_update_noalloc_rejects_too_many_sites():
    torch = pytest.importorskip("torch")
    n = L.UPDATE_NOALLOC_MAX_SITES + 1
    cell = torch.zeros((1, 1, 64), dtype=torch.int32, device="cuda")
    sites = torch.zeros(n, dtype=torch.int32, device="cuda")
    with pytest.raises(L.LsrvtError) as e:
        L.lsrvt_update_noalloc(cell, sites)
    assert e.value.code == L.ELIMIT
