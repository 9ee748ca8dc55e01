"""Independent brute-force references used to pin the oracle.

Each routine reaches the same result as the oracle by a different route:
library routines (numpy searchsorted, scipy.ndimage.label, scipy.sparse.csgraph
shortest paths), exhaustive enumeration, or exact rationals.  None of them
calls the oracle or the GPU library.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
from scipy import ndimage
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import shortest_path

NONE_ID = 0xFFFFFFFF


def bands_searchsorted(f, iso):
    """#{i : iso_i < f} == numpy.searchsorted(iso, f, side='left')."""
    return np.searchsorted(np.asarray(iso, dtype=np.float32), np.asarray(f, dtype=np.float32),
                           side="left").astype(np.uint8)


def components_scipy(band, n_bands):
    """Canonical component ids from scipy.ndimage.label run on each band.

    Components are ordered by (band, smallest linear index)."""
    struct = ndimage.generate_binary_structure(3, 1)
    flat = band.ravel()
    n = flat.size
    entries = []  # (band, min index, mask-label) per component
    labels_all = []
    for b in range(n_bands):
        lab, k = ndimage.label(band == b, structure=struct)
        labels_all.append(lab.ravel())
        if k == 0:
            continue
        lf = lab.ravel()
        idx = np.nonzero(lf)[0]
        mins = np.full(k + 1, n, dtype=np.int64)
        np.minimum.at(mins, lf[idx], idx)
        for lbl in range(1, k + 1):
            entries.append((b, int(mins[lbl]), lbl))
    entries.sort()
    comp = np.empty(n, dtype=np.uint32)
    for cid, (b, _, lbl) in enumerate(entries):
        comp[labels_all[b] == lbl] = cid
    sizes = np.bincount(comp, minlength=len(entries)).astype(np.uint64)
    first = np.array([e[1] for e in entries], dtype=np.uint32)
    cb = np.array([e[0] for e in entries], dtype=np.uint8)
    bo = np.zeros(n_bands + 1, dtype=np.uint32)
    np.add.at(bo, cb.astype(np.int64) + 1, 1)
    bo = np.cumsum(bo).astype(np.uint32)
    return comp.reshape(band.shape), len(entries), cb, sizes, first, bo


def components_unionfind(band):
    """Union-find over every same-band face edge; canonical (band, min index) ids."""
    nz, ny, nx = band.shape
    n = band.size
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    flat = band.ravel()
    for v in range(n):
        x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
        for (dx, dy, dz) in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
            if x + dx < nx and y + dy < ny and z + dz < nz:
                w = v + dx + nx * dy + nx * ny * dz
                if flat[w] == flat[v]:
                    ra, rb = find(v), find(w)
                    if ra != rb:
                        parent[max(ra, rb)] = min(ra, rb)
    roots = sorted({find(v) for v in range(n)}, key=lambda r: (flat[r], r))
    rid = {r: i for i, r in enumerate(roots)}
    return np.array([rid[find(v)] for v in range(n)], dtype=np.uint32).reshape(band.shape)


def adjacency(comp):
    """Sparse adjacency of the 6-neighbour graph restricted to equal labels."""
    nz, ny, nx = comp.shape
    idx = np.arange(comp.size).reshape(comp.shape)
    rows, cols = [], []
    for axis in range(3):
        a = [slice(None)] * 3
        b = [slice(None)] * 3
        a[axis] = slice(0, -1)
        b[axis] = slice(1, None)
        same = comp[tuple(a)] == comp[tuple(b)]
        rows.append(idx[tuple(a)][same])
        cols.append(idx[tuple(b)][same])
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    n = comp.size
    m = coo_matrix((np.ones(len(r)), (r, c)), shape=(n, n))
    return (m + m.T).tocsr()


def vt_allpairs(comp, sites):
    """Eq. 1 by brute force: all-pairs hop distances, then the lexicographic
    argmin of (distance, site id) per voxel."""
    n = comp.size
    sites = np.asarray(sites, dtype=np.int64)
    if len(sites) == 0:
        return np.full(comp.shape, NONE_ID, dtype=np.uint32), np.full(comp.shape, np.inf)
    D = shortest_path(adjacency(comp), method="D", unweighted=True, directed=False, indices=sites)
    cell = np.full(n, NONE_ID, dtype=np.uint32)
    dist = np.full(n, np.inf)
    for v in range(n):
        best = None
        for s in range(len(sites)):
            d = D[s, v]
            if np.isinf(d):
                continue
            if best is None or (d, s) < best:
                best = (d, s)
        if best is not None:
            dist[v] = best[0]
            cell[v] = best[1]
    return cell.reshape(comp.shape), dist.reshape(comp.shape)


def update_fraction(cell, sites, weights=None):
    """Site update with exact rationals: centroid c = sum w x / sum w, then the
    in-cell voxel minimising |x - c|^2, ties to the lower linear index."""
    nz, ny, nx = cell.shape
    flat = cell.ravel()
    w = np.ones(flat.size, dtype=np.int64) if weights is None else np.asarray(weights).ravel().astype(np.int64)
    out = np.array(sites, dtype=np.uint32, copy=True)
    for s in range(len(sites)):
        vox = np.nonzero(flat == s)[0]
        M = int(w[vox].sum()) if len(vox) else 0
        if M == 0:
            continue
        coords = [(int(v % nx), int((v // nx) % ny), int(v // (nx * ny))) for v in vox]
        c = [Fraction(sum(int(w[v]) * co[a] for v, co in zip(vox, coords)), M) for a in range(3)]
        best = None
        for v, co in zip(vox, coords):
            d2 = sum((co[a] - c[a]) ** 2 for a in range(3))
            if best is None or d2 < best[0] or (d2 == best[0] and v < best[1]):
                best = (d2, int(v))
        out[s] = best[1]
    return out


def stats_numpy(unit, n_units, variables, edges=None, cov=False):
    """Per-unit statistics with numpy: bincount sums, np.var-style centred sums,
    minimum/maximum.at, and searchsorted(side='right') over the interior edges."""
    u = np.asarray(unit).ravel().astype(np.int64)
    keep = u != NONE_ID
    u = u[keep]
    m = variables.shape[0]
    x = variables.reshape(m, -1)[:, keep].astype(np.float64)
    n = np.bincount(u, minlength=n_units).astype(np.uint64)
    mean = np.zeros((n_units, m))
    m2 = np.zeros((n_units, m))
    vmin = np.full((n_units, m), np.inf, dtype=np.float32)
    vmax = np.full((n_units, m), -np.inf, dtype=np.float32)
    nz = n > 0
    for j in range(m):
        s = np.bincount(u, weights=x[j], minlength=n_units)
        mean[nz, j] = s[nz] / n[nz]
        d = x[j] - mean[u, j]
        m2[:, j] = np.bincount(u, weights=d * d, minlength=n_units)
        xf = variables.reshape(m, -1)[j, keep]
        np.minimum.at(vmin[:, j], u, xf)
        np.maximum.at(vmax[:, j], u, xf)
    hist = None
    if edges is not None:
        B = edges.shape[1] - 1
        hist = np.zeros((n_units, m, B), dtype=np.uint32)
        for j in range(m):
            b = np.searchsorted(edges[j, 1:B], variables.reshape(m, -1)[j, keep], side="right")
            np.add.at(hist[:, j, :], (u, b), 1)
    cv = None
    if cov:
        P = m * (m + 1) // 2
        cv = np.zeros((n_units, P))
        p = 0
        for j in range(m):
            dj = x[j] - mean[u, j]
            for k in range(j, m):
                dk = x[k] - mean[u, k]
                cv[:, p] = np.bincount(u, weights=dj * dk, minlength=n_units)
                p += 1
    return n, mean, m2, vmin, vmax, hist, cv


def random_bands(shape, n_bands, rng, smooth=False):
    """Random band labels; ``smooth`` makes larger, more contorted components."""
    if smooth:
        f = rng.normal(size=shape)
        f = ndimage.uniform_filter(f, size=3, mode="wrap")
        qs = np.quantile(f, np.linspace(0, 1, n_bands + 1)[1:-1])
        return np.searchsorted(qs, f).astype(np.uint8)
    return rng.integers(0, n_bands, size=shape).astype(np.uint8)
