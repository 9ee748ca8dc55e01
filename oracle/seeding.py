"""Oracle for the stratified initial sites (Sec. 3.2.1, Eq. 3 and Eq. 4).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy and Python
integers; every quantity that decides an integer is computed exactly.

What is computed (the readings of the printed formulas are listed with each
step):

1. Voxel mass m(v) = lut[w(v)] (the attraction gamma enters only through the
   caller's table, e.g. round(s * w^gamma)); m = w without a table and m = 1
   without weights.
2. Component mass m(C) = sum of m(v) over C, total mass M = sum over all voxels.
3. Sites per component (Eq. 3): with rho voxels per site,
   n_c = max(ceil(m(C) * N / (rho * M)), 1) -- the printed form reduces to the
   site density alpha; here the density is one site per rho voxels of average
   mass.  A component of zero mass gets one site, its first voxel.
4. Blocks: the volume is cut into cubes of edge `block`; the blocks of a
   component are its (component, block) pairs, ordered by block index.
   Each gets floor(n_c * m(b) / m(C)) sites; the n_c - sum of those that
   remain go one each to the blocks with the largest remainders
   n_c * m(b) mod m(C), ties to the lower block index (Eq. 4's "most
   under-represented blocks"; as printed ur(b) does not depend on the block).
5. Placement inside a (component, block) pair with n_b sites: systematic
   sampling proportional to mass over the pair's voxels in linear-index
   order.  With o uniform in [0, m(b)) the points are
   p_j = floor((o + j m(b)) / n_b), j = 0 .. n_b - 1, and site j is the voxel
   whose cumulative-mass interval [C_{i-1}, C_i) holds p_j (a voxel heavier
   than m(b) / n_b can be picked twice: co-located sites are allowed).
   o = (lo | hi << 32) mod m(b), where (lo, hi) are the first two words of
   Philox4x32-10 with key (seed low, seed high) and counter
   (block, component, 0, 0).
6. Sites are numbered by (component, block, j).
"""
from __future__ import annotations

import numpy as np

NONE_ID = 0xFFFFFFFF

# Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): multipliers and Weyl
# key increments of the published definition.
_PHILOX_M0 = 0xD2511F53
_PHILOX_M1 = 0xCD9E8D57
_PHILOX_W0 = 0x9E3779B9
_PHILOX_W1 = 0xBB67AE85
_MASK32 = 0xFFFFFFFF


def philox4x32(counter, key, rounds: int = 10):
    """Philox4x32 with `rounds` rounds on a 4-word counter and a 2-word key."""
    c0, c1, c2, c3 = (int(v) & _MASK32 for v in counter)
    k0, k1 = (int(v) & _MASK32 for v in key)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + _PHILOX_W0) & _MASK32
            k1 = (k1 + _PHILOX_W1) & _MASK32
        p0 = _PHILOX_M0 * c0
        p1 = _PHILOX_M1 * c2
        hi0, lo0 = p0 >> 32, p0 & _MASK32
        hi1, lo1 = p1 >> 32, p1 & _MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & _MASK32, lo1, (hi0 ^ c3 ^ k1) & _MASK32, lo0
    return c0, c1, c2, c3


def pair_offset(seed: int, block: int, comp: int, mass: int) -> int:
    """The systematic-sampling offset o in [0, mass) of one (component, block) pair."""
    w = philox4x32((block, comp, 0, 0), (seed & _MASK32, (seed >> 32) & _MASK32))
    return (w[0] | (w[1] << 32)) % mass


def voxel_mass(weights, lut, n: int) -> np.ndarray:
    """m(v) as Python-int-safe int64 (every value < 2^32)."""
    if weights is None:
        return np.ones(n, dtype=np.int64)
    w = np.asarray(weights).reshape(-1).astype(np.int64)
    if lut is None:
        return w
    return np.asarray(lut, dtype=np.int64)[w]


def block_index(shape, block: int) -> np.ndarray:
    """Block of every voxel (cubes of edge `block`, x fastest)."""
    nz, ny, nx = shape
    nbx, nby = -(-nx // block), -(-ny // block)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((x // block) + nbx * ((y // block) + nby * (z // block))).reshape(-1).astype(np.int64)


def sites_per_component(comp_mass, n_voxels: int, total_mass: int, rho: int):
    """Eq. 3 as read above: n_c = max(ceil(m(C) N / (rho M)), 1), exact."""
    out = []
    den = rho * total_mass
    for mc in comp_mass:
        mc = int(mc)
        n = -(-(mc * n_voxels) // den) if den else 0
        out.append(max(n, 1))
    return out


def apportion(n_c: int, masses, blocks):
    """Eq. 4 as read above: floor shares plus largest remainders (ties to the lower block)."""
    mc = sum(int(m) for m in masses)
    base = [(n_c * int(m)) // mc for m in masses]
    rem = [(n_c * int(m)) % mc for m in masses]
    left = n_c - sum(base)
    order = sorted(range(len(masses)), key=lambda i: (-rem[i], int(blocks[i])))
    for i in order[:left]:
        base[i] += 1
    return base


def seed_stratified(comp: np.ndarray, n_comp: int, weights=None, lut=None, rho: int = 4096, block: int = 16,
                    seed: int = 0):
    """Initial sites (linear indices, uint32) numbered by (component, block, j)."""
    shape = comp.shape
    c = np.asarray(comp).reshape(-1).astype(np.int64)
    n = c.size
    if n == 0:
        return np.zeros(0, dtype=np.uint32)
    m = voxel_mass(weights, lut, n)
    blk = block_index(shape, block)
    total = int(m.sum())
    comp_mass = _exact_sums(c, m, n_comp)
    n_sites = sites_per_component(comp_mass, n, total, rho)
    # (component, block) pairs, ordered by component then block; voxels of a pair in linear order
    key = c * (int(blk.max()) + 1 if n else 1) + blk
    order = np.argsort(key, kind="stable")
    sites = []
    i = 0
    first_voxel = np.full(n_comp, -1, dtype=np.int64)
    uc, ui = np.unique(c, return_index=True)  # first occurrence = smallest linear index
    first_voxel[uc] = ui
    cs = c[order]
    comp_end = np.concatenate((np.flatnonzero(np.diff(cs)) + 1, [n]))
    for j in comp_end:
        j = int(j)
        cc = int(cs[i])
        seg = order[i:j]  # voxels of component cc, by block then linear index
        if comp_mass[cc] == 0:
            sites.append(int(first_voxel[cc]))
            i = j
            continue
        bl = blk[seg]
        starts = [0] + [int(k) for k in np.flatnonzero(np.diff(bl)) + 1] + [len(seg)]
        pair_vox = [seg[starts[k]:starts[k + 1]] for k in range(len(starts) - 1)]
        pair_blk = [int(blk[p[0]]) for p in pair_vox]
        pair_mass = [int(m[p].sum()) for p in pair_vox]
        nb = apportion(n_sites[cc], pair_mass, pair_blk)
        for p, b, mb, k in zip(pair_vox, pair_blk, pair_mass, nb):
            if k == 0:
                continue
            o = pair_offset(seed, b, cc, mb)
            cum = np.cumsum(m[p])
            for t in range(k):
                pt = (o + t * mb) // k
                sites.append(int(p[int(np.searchsorted(cum, pt, side="right"))]))
        i = j
    return np.asarray(sites, dtype=np.uint32)


def _exact_sums(c: np.ndarray, m: np.ndarray, n_comp: int):
    """Per-component sums of m as Python ints (exact for any size)."""
    out = [0] * n_comp
    order = np.argsort(c, kind="stable")
    cs = c[order]
    ms = m[order]
    bounds = np.flatnonzero(np.diff(cs)) + 1
    starts = np.concatenate(([0], bounds))
    ends = np.concatenate((bounds, [cs.size]))
    for s, e in zip(starts, ends):
        if e > s:
            out[int(cs[s])] = int(ms[s:e].sum())
    return out
