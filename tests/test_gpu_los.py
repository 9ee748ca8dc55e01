"""The line-of-sight tessellation, site update and Lloyd loop on the GPU
(lsrvt_los_vt, lsrvt_los_update, lsrvt_los_cvt) against the oracle.

Both sides compute path lengths as sqrt of exact integers (correctly
rounded) plus float64 sums in the same order, compare them with the same
margins and do the site update in exact integers, so every output is
compared bit for bit: lengths, sources, phi, cells, the sweep counts of both
stages, site positions, anchors and targets.  At 256^3 the oracle's sweeps
are too slow, so the result is checked through properties that hold at any
size (the fixed point of the sweeps, clear segments, phi and cells) and,
per site, against the oracle's exact target and clamped move."""
import numpy as np
import pytest

import oracle
import paper_2208_06970_amd as L
import synth
from tests.gpu_util import banner, dev, host

pytestmark = pytest.mark.gpu
NONE = oracle.NONE_ID
SITE = oracle.SITE_FLAG


def _field_case(shape, seed, n_iso, rho):
    f = synth.fourier_field(shape, seed, n_modes=64)
    iso = synth.quantile_isovalues(f, [(i + 1) / (n_iso + 1) for i in range(n_iso)])
    band = oracle.bands(f, iso)
    cc = oracle.components(band, n_iso + 1)
    w = synth.gradient_weight(f)
    seeds = synth.seed_sites(cc.comp, cc.n_comp, w, rho, seed)
    return cc.comp, w, seeds


def _q8(seeds, shape, seed, corners=False):
    nz, ny, nx = shape
    s = seeds.astype(np.int64)
    q = np.stack([s % nx, (s // nx) % ny, s // (nx * ny)], axis=1) * 256
    rng = np.random.default_rng(seed)
    off = rng.choice([-128, 0, 128], q.shape) if corners else rng.integers(-128, 129, q.shape)
    for i, n in enumerate((nx, ny, nz)):  # stay inside the volume
        off[:, i] = np.where((q[:, i] // 256 == 0) & (off[:, i] < 0), 0, off[:, i])
        off[:, i] = np.where((q[:, i] // 256 == n - 1) & (off[:, i] > 0), 0, off[:, i])
    return (q + off).astype(np.int32)


def _cmp_vt(got, want):
    np.testing.assert_array_equal(host(got.dist), want.dist)
    np.testing.assert_array_equal(host(got.src, np.uint32), want.src)
    np.testing.assert_array_equal(host(got.phi, np.uint32), want.phi)
    np.testing.assert_array_equal(host(got.cell, np.uint32), want.cell)
    assert got.sweeps == want.sweeps


@pytest.mark.parametrize("shape,seed,n_iso,rho,corners", [
    ((40, 36, 44), 1, 3, 300.0, False),
    ((33, 48, 29), 2, 5, 150.0, True),
    ((20, 64, 70), 3, 2, 900.0, False),
])
def test_los_vt_and_update_match_oracle(shape, seed, n_iso, rho, corners):
    comp, w, seeds = _field_case(shape, seed, n_iso, rho)
    q = _q8(seeds, shape, seed, corners)
    banner(f"los_vt: {shape} S={len(seeds)}")
    want = oracle.los_vt(comp, q, seeds)
    d_comp, d_q, d_a = dev(comp), dev(q), dev(seeds)
    got = L.lsrvt_los_vt(d_comp, d_q, d_a)
    _cmp_vt(got, want)
    los = np.mean(want.src[comp != NONE] & SITE != 0)
    print(f"sweeps {want.sweeps}, line-of-sight fraction {los:.3f}")
    banner(f"los_update: {shape}")
    wq, wa, wt = oracle.los_update(comp, want.cell, want.phi, q, seeds, w)
    tg = L.lsrvt_los_update(d_comp, got.cell, got.phi, d_q, d_a, dev(w))
    np.testing.assert_array_equal(host(tg), wt)
    np.testing.assert_array_equal(host(d_q), wq)
    np.testing.assert_array_equal(host(d_a, np.uint32), wa)
    assert np.any(wq != q), "some site should move"


@pytest.mark.parametrize("shape,seed,iters,weighted", [
    ((36, 40, 38), 4, 3, True),
    ((24, 30, 66), 5, 2, False),
])
def test_los_cvt_matches_oracle(shape, seed, iters, weighted):
    comp, w, seeds = _field_case(shape, seed, 4, 250.0)
    w = w if weighted else None
    banner(f"los_cvt: {shape} iters={iters}")
    want = oracle.los_cvt(comp, seeds, w, iters)
    got = L.lsrvt_los_cvt(dev(comp), dev(seeds), None if w is None else dev(w), iters)
    np.testing.assert_array_equal(host(got.site_q), want.site_q)
    np.testing.assert_array_equal(host(got.anchor, np.uint32), want.anchor)
    np.testing.assert_array_equal(host(got.vt.dist), want.dist)
    np.testing.assert_array_equal(host(got.vt.src, np.uint32), want.src)
    np.testing.assert_array_equal(host(got.vt.phi, np.uint32), want.phi)
    np.testing.assert_array_equal(host(got.vt.cell, np.uint32), want.cell)


def test_los_edge_cases():
    shape = (6, 7, 9)
    # no sites: nothing is reached
    comp = np.zeros(shape, dtype=np.uint32)
    comp[2] = NONE
    banner("los edge: no sites")
    z = dev(np.zeros((0, 3), dtype=np.int32))
    r = L.lsrvt_los_vt(dev(comp), z, dev(np.zeros(0, dtype=np.uint32)))
    assert np.all(np.isinf(host(r.dist))) and np.all(host(r.src, np.uint32) == NONE)
    assert np.all(host(r.cell, np.uint32) == NONE)
    # co-located sites share an anchor (the lower id holds it); a one-voxel
    # component; a site on a corner of its anchor; a component with no site
    comp = np.zeros(shape, dtype=np.uint32)
    comp[:, :, 4] = NONE                  # wall: x < 4 is component 0, x > 4 component 1 ...
    comp[:, :, 5:] = 1
    comp[3, 3, 7] = 2                     # ... with a one-voxel component 2 inside it
    comp[0, 0, 0] = 3                     # and a one-voxel component 3 that gets no site
    lin = lambda x, y, zz: x + 9 * (y + 7 * zz)
    seeds = np.array([lin(1, 1, 1), lin(1, 1, 1), lin(6, 2, 4), lin(7, 3, 3), lin(2, 5, 5)], dtype=np.uint32)
    q = _q8(seeds, shape, 0)
    q[1] = q[0]
    q[4] = [2 * 256 + 128, 5 * 256 - 128, 5 * 256 + 128]   # a corner of its anchor, on the volume's face
    banner("los edge: co-located, single voxel, corner")
    want = oracle.los_vt(comp, q, seeds)
    got = L.lsrvt_los_vt(dev(comp), dev(q), dev(seeds))
    _cmp_vt(got, want)
    assert not np.any(want.cell == 1)
    assert want.cell[3, 3, 7] == 3 and want.cell[0, 0, 0] == NONE
    w = np.full(shape, 3, dtype=np.uint16)
    wq, wa, wt = oracle.los_update(comp, want.cell, want.phi, q, seeds, w)
    d_q, d_a = dev(q), dev(seeds)
    tg = L.lsrvt_los_update(dev(comp), got.cell, got.phi, d_q, d_a, dev(w))
    np.testing.assert_array_equal(host(tg), wt)
    np.testing.assert_array_equal(host(d_q), wq)
    np.testing.assert_array_equal(host(d_a, np.uint32), wa)
    assert np.all(wt[1] == np.iinfo(np.int32).min)   # the losing co-located site has no cell
    # an anchor that does not hold its site is refused
    bad = q.copy()
    bad[0, 0] += 200
    with pytest.raises(L.LsrvtError):
        L.lsrvt_los_vt(dev(comp), dev(bad), dev(seeds))


def test_los_fullsize_properties():
    """The 256^3 benchmark field: two Lloyd updates, then the fixed point of
    the final tessellation, its paths, phi and cells; per site the exact
    target and a sample of clamped moves against the oracle."""
    wl = synth.fourier_workload()
    band = oracle.bands(wl.field, wl.iso)
    cc = oracle.components(band, wl.n_bands)
    seeds = synth.workload_sites(wl, cc.comp, cc.n_comp)
    comp = cc.comp
    nz, ny, nx = comp.shape
    d_comp, d_w = dev(comp), dev(wl.weights)
    banner(f"los_cvt: 256^3, S={len(seeds)}, 2 updates")
    res = L.lsrvt_los_cvt(d_comp, dev(seeds), d_w, 2)
    print(f"sweeps in 3 passes: {res.vt.sweeps[0]}")
    d = host(res.vt.dist).ravel()
    src = host(res.vt.src, np.uint32).ravel()
    phi = host(res.vt.phi, np.uint32).ravel()
    cell = host(res.vt.cell, np.uint32).ravel()
    q = host(res.site_q).astype(np.int64)
    a = host(res.anchor, np.uint32).astype(np.int64)
    cf = comp.ravel()
    lab = cf != NONE
    # every component that holds a site is covered; nothing else is
    has_site = np.zeros(cc.n_comp, dtype=bool)
    has_site[cf[a]] = True
    reach = np.zeros(cf.shape, dtype=bool)
    reach[lab] = has_site[cf[lab]]
    assert np.array_equal(src != NONE, reach)
    v = np.flatnonzero(reach)
    x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
    # line-of-sight voxels: the exact leg to their site
    los = (src[v] & SITE) != 0
    s = (src[v][los] & (SITE - 1)).astype(np.int64)
    n2 = (256 * x[los] - q[s, 0]) ** 2 + (256 * y[los] - q[s, 1]) ** 2 + (256 * z[los] - q[s, 2]) ** 2
    assert np.array_equal(d[v][los], np.sqrt(n2.astype(np.float64)) / 256.0)
    # other voxels: their length is the leg to the source plus its length
    u = src[v][~los].astype(np.int64)
    leg = np.sqrt(((x[~los] - u % nx) ** 2 + (y[~los] - (u // nx) % ny) ** 2
                   + (z[~los] - u // (nx * ny)) ** 2).astype(np.float64))
    tot = leg + d[u]
    dv = d[v][~los]
    assert np.all(dv >= tot) and np.all(dv <= tot * (1 + 2.0 ** -39))
    # the fixed point: no face neighbour offers a path shorter by the margin
    dd = d.reshape(comp.shape)
    for ax in range(3):
        for sh in (1, -1):
            nbd = np.roll(dd, sh, axis=ax)
            nbc = np.roll(comp, sh, axis=ax)
            edge = np.zeros(comp.shape, dtype=bool)
            sl = [slice(None)] * 3
            sl[ax] = 0 if sh == 1 else -1
            edge[tuple(sl)] = True
            ok = (~reach.reshape(comp.shape)) | (nbc != comp) | edge | (dd <= (nbd + 1.0) * (1 + 2.0 ** -39))
            assert np.all(ok)
    # phi and cells
    assert np.all((src[phi[v]] & SITE) != 0)
    assert np.array_equal(cell[v], src[phi[v]] & (SITE - 1))
    # a sample of segments is clear
    rng = np.random.default_rng(1)
    for i in rng.choice(len(v), 300, replace=False):
        vv = int(v[i])
        t = int(a[src[vv] & (SITE - 1)]) if src[vv] & SITE else int(src[vv])
        p0 = (vv % nx, (vv // nx) % ny, vv // (nx * ny))
        p1 = (t % nx, (t // nx) % ny, t // (nx * ny))
        cov = oracle.supercover(p0, p1)
        assert np.all(comp[cov[:, 2], cov[:, 1], cov[:, 0]] == cf[vv])
    # the update: exact targets for every site, and the clamped move of a
    # sample of sites, against the oracle
    banner("los_update: 256^3")
    q0 = res.site_q.clone()
    a0 = res.anchor.clone()
    tg = host(L.lsrvt_los_update(d_comp, res.vt.cell, res.vt.phi, res.site_q, res.anchor, d_w)).astype(np.int64)
    wv = wl.weights.ravel().astype(np.int64)
    S = len(seeds)
    px, py, pz = phi[v] % nx, (phi[v] // nx) % ny, phi[v] // (nx * ny)
    # exact integer sums: int64 suffices (< 2^62 under the size limits)
    m_int = np.zeros(S, dtype=np.int64)
    np.add.at(m_int, cell[v], wv[v])
    sx = np.zeros((S, 3), dtype=np.int64)
    for i, p in enumerate((px, py, pz)):
        np.add.at(sx[:, i], cell[v], wv[v] * p.astype(np.int64))
    for s_ in range(S):
        if m_int[s_] == 0:
            assert np.all(tg[s_] == np.iinfo(np.int32).min)
            continue
        for i in range(3):
            qq, r = divmod(int(sx[s_, i]), int(m_int[s_]))
            assert tg[s_, i] == 256 * qq + (512 * r + int(m_int[s_])) // (2 * int(m_int[s_]))
    nq = host(res.site_q)
    na = host(res.anchor, np.uint32)
    q0h, a0h = host(q0), host(a0, np.uint32)
    for s_ in rng.choice(S, 400, replace=False):
        if m_int[s_] == 0:
            continue
        wx, wa_ = oracle.los_clamp(comp, q0h[s_], int(a0h[s_]), tg[s_])
        assert np.array_equal(nq[s_], wx) and na[s_] == wa_, s_


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 37), (1, 23, 1), (5, 1, 9), (3, 70, 2)])
def test_los_degenerate_shapes(shape):
    """One voxel, lines along x and y, one-voxel-thick slabs: the walks and
    neighbour checks at every face of the volume."""
    rng = np.random.default_rng(sum(shape))
    n = int(np.prod(shape))
    comp = np.where(rng.random(shape) < 0.15, NONE, rng.integers(0, 2, shape)).astype(np.uint32)
    if n == 1:
        comp[...] = 0
    cand = np.flatnonzero(comp.ravel() != NONE)
    seeds = np.sort(rng.choice(cand, min(len(cand), 3), replace=False)).astype(np.uint32)
    w = rng.integers(1, 9, shape).astype(np.uint16)
    banner(f"los degenerate: {shape} S={len(seeds)}")
    want = oracle.los_cvt(comp, seeds, w, 3)
    got = L.lsrvt_los_cvt(dev(comp), dev(seeds), dev(w), 3)
    np.testing.assert_array_equal(host(got.site_q), want.site_q)
    np.testing.assert_array_equal(host(got.anchor, np.uint32), want.anchor)
    np.testing.assert_array_equal(host(got.vt.dist), want.dist)
    np.testing.assert_array_equal(host(got.vt.src, np.uint32), want.src)
    np.testing.assert_array_equal(host(got.vt.cell, np.uint32), want.cell)


def test_los_update_every_voxel_a_site():
    """More distinct cells per 64x8x8 tile than the Eq. 2 sums' LDS table
    holds (512): every voxel a site, so the global-atomic fallback runs;
    bit-exact against the oracle."""
    shape = (12, 20, 70)
    comp = np.zeros(shape, dtype=np.uint32)
    comp[:, :, 35:] = 1
    rng = np.random.default_rng(17)
    seeds = rng.permutation(comp.size).astype(np.uint32)
    w = rng.integers(1, 65536, size=shape).astype(np.uint16)
    q = _q8(seeds, shape, 17)
    banner("los_update: every voxel a site")
    want = oracle.los_vt(comp, q, seeds)
    d_comp, d_q, d_a = dev(comp), dev(q), dev(seeds)
    got = L.lsrvt_los_vt(d_comp, d_q, d_a)
    _cmp_vt(got, want)
    wq, wa, wt = oracle.los_update(comp, want.cell, want.phi, q, seeds, w)
    tg = L.lsrvt_los_update(d_comp, got.cell, got.phi, d_q, d_a, dev(w))
    np.testing.assert_array_equal(host(tg), wt)
    np.testing.assert_array_equal(host(d_q), wq)
    np.testing.assert_array_equal(host(d_a, np.uint32), wa)
