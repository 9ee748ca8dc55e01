"""CPU oracle for the level-set restricted geodesic Voronoi pipeline.

TEST INFRASTRUCTURE ONLY.  This package is the plain reference the GPU library
is checked against.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the GPU library never imports it and it
imports nothing from the GPU library.

The arithmetic lives in ``lsrvt_oracle.c`` (plain C, double precision, exact
integers for the site update); this module only marshals numpy arrays through
ctypes.  Each function cites the passage of the paper it follows:

* :func:`bands`       -- Sec. 3.1, isoband definition B_{a,b} = {a < f <= b}
* :func:`components`  -- Sec. 3.1, connected components of each isoband,
  numbered by (band, smallest member index) as in the hierarchical layout of
  Sec. 3.2.4 / Fig. 5
* :func:`vt`          -- Eq. 1, restricted geodesic Voronoi regions (hop
  distance in the restricted 6-neighbour graph, ties to the lower site id)
* :func:`update`      -- Sec. 3.1 "Centroids", weighted centre of mass moved
  to the nearest in-region voxel
* :func:`cvt`         -- Algorithm 1 with a fixed number of updates
* :func:`stats`       -- Sec. 3.3 "Aggregation": per-unit moments, extrema,
  histograms and covariance, computed directly per unit in double precision
* :func:`chan_merge`  -- pairwise merge of (n, mean, M2, C) summaries, used by
  the tests to check that merged cell statistics equal the direct ones
* :func:`layout`      -- Sec. 3.2.4 "Data Reduction and Structured Data
  Layout" / Fig. 5: the voxels of the cells ordered by band, component and
  cell, with offsets per cell, component and band (numpy, stable sorts)
* :func:`extract`     -- the raw variables in that order
* :func:`comoments`   -- Sec. 4.4: centred joint moments of orders 2-4 of
  every unit, direct two-pass float64 numpy (in ``moments.py``)
* :func:`los_vt`, :func:`los_update`, :func:`los_cvt` -- Eq. 1 with the
  Euclidean line-of-sight paths of Sec. 3.2.2, the Eq. 2 centroid with
  masses carried to line-of-sight voxels and the ray-clamped move of
  Sec. 3.2.3 (in ``los_oracle.c``), with :func:`supercover`, the voxels a
  segment between two voxel centres touches
* :func:`seed_stratified` -- Sec. 3.2.1, Eq. 3 and Eq. 4: stratified initial
  sites (numpy and exact Python integers, in ``seeding.py``, with the
  Philox4x32-10 generator it draws from)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "lsrvt_oracle.c"), os.path.join(_HERE, "los_oracle.c")]
_LIB = os.path.join(_HERE, "liblsrvt_oracle.so")

NONE_ID = 0xFFFFFFFF
OK, EINVAL, ENAN, ENOMEM, ELIMIT = 0, 1, 2, 3, 4


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fused multiply-add contraction)."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f) for f in _SRCS)
    if force or stale:
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
             "-o", tmp, *_SRCS, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        lib.oracle_bands.argtypes = [P, i64, P, i32, P]
        lib.oracle_components.argtypes = [P, i32, i32, i32, i32, P, P, P, P, P, P]
        lib.oracle_vt.argtypes = [P, i32, i32, i32, P, u32, P, P]
        lib.oracle_vt_unpruned.argtypes = [P, i32, i32, i32, P, u32, P, P]
        lib.oracle_update.argtypes = [P, i32, i32, i32, P, P, u32, P]
        lib.oracle_cvt.argtypes = [P, i32, i32, i32, P, u32, P, i32, P, P, P, P]
        lib.oracle_stats.argtypes = [P, i64, u32, P, i32, P, i32, P, P, P, P, P, P, P]
        lib.oracle_supercover.argtypes = [P, P, P, i64]
        lib.oracle_supercover.restype = i64
        lib.oracle_los_vt.argtypes = [P, i32, i32, i32, P, P, u32, P, P, P, P, P]
        lib.oracle_los_update.argtypes = [P, i32, i32, i32, P, P, P, u32, P, P, P]
        lib.oracle_los_cvt.argtypes = [P, i32, i32, i32, P, u32, P, i32, P, P, P, P, P, P]
        lib.oracle_los_clamp.argtypes = [P, i32, i32, i32, P, P, P]
        for f in (lib.oracle_bands, lib.oracle_components, lib.oracle_vt, lib.oracle_vt_unpruned,
                  lib.oracle_update, lib.oracle_cvt, lib.oracle_stats, lib.oracle_los_vt,
                  lib.oracle_los_update, lib.oracle_los_cvt, lib.oracle_los_clamp):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dims(shape):
    nz, ny, nx = (int(s) for s in shape)
    return nx, ny, nz


def _check(code, what):
    if code != OK:
        raise OracleError(code, what)


# --------------------------------------------------------------------------
def bands(field: np.ndarray, iso) -> np.ndarray:
    """Band index #{i : iso_i < f(v)} per voxel (Sec. 3.1).  Raises on NaN."""
    f = np.ascontiguousarray(field, dtype=np.float32)
    iso = np.ascontiguousarray(iso, dtype=np.float32)
    out = np.empty(f.shape, dtype=np.uint8)
    _check(_load().oracle_bands(_ptr(f), f.size, _ptr(iso), len(iso), _ptr(out)), "bands")
    return out


@dataclass
class Components:
    comp: np.ndarray        # uint32[nz, ny, nx]
    n_comp: int
    comp_band: np.ndarray   # uint8[n_comp]
    comp_size: np.ndarray   # uint64[n_comp]
    comp_first: np.ndarray  # uint32[n_comp]
    band_offset: np.ndarray  # uint32[n_bands + 1]


def components(band: np.ndarray, n_bands: int) -> Components:
    """6-connected components of each isoband, numbered by (band, min index)."""
    b = np.ascontiguousarray(band, dtype=np.uint8)
    nx, ny, nz = _dims(b.shape)
    n = b.size
    comp = np.empty(b.shape, dtype=np.uint32)
    ncomp = np.zeros(1, dtype=np.uint32)
    cb = np.empty(n, dtype=np.uint8)
    cs = np.empty(n, dtype=np.uint64)
    cf = np.empty(n, dtype=np.uint32)
    bo = np.empty(n_bands + 1, dtype=np.uint32)
    _check(_load().oracle_components(_ptr(b), nx, ny, nz, n_bands, _ptr(comp), _ptr(ncomp),
                                     _ptr(cb), _ptr(cs), _ptr(cf), _ptr(bo)), "components")
    k = int(ncomp[0])
    return Components(comp, k, cb[:k].copy(), cs[:k].copy(), cf[:k].copy(), bo)


def vt(comp: np.ndarray, sites, pruned: bool = True, return_dist: bool = False):
    """Restricted geodesic Voronoi regions of Eq. 1 (hop metric, id tie-break)."""
    c = np.ascontiguousarray(comp, dtype=np.uint32)
    s = np.ascontiguousarray(sites, dtype=np.uint32)
    nx, ny, nz = _dims(c.shape)
    cell = np.empty(c.shape, dtype=np.uint32)
    dist = np.empty(c.shape, dtype=np.uint32)
    fn = _load().oracle_vt if pruned else _load().oracle_vt_unpruned
    _check(fn(_ptr(c), nx, ny, nz, _ptr(s), len(s), _ptr(cell), _ptr(dist)), "vt")
    return (cell, dist) if return_dist else cell


def update(cell: np.ndarray, sites, weights=None):
    """One site update: exact weighted centroid snapped to the nearest in-cell voxel.

    Returns (new_sites, ds) where ds[s] is the Euclidean move of site s."""
    c = np.ascontiguousarray(cell, dtype=np.uint32)
    nx, ny, nz = _dims(c.shape)
    s = np.array(sites, dtype=np.uint32, copy=True)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.uint16)
    ds = np.zeros(len(s), dtype=np.float64)
    _check(_load().oracle_update(_ptr(c), nx, ny, nz, _ptr(w), _ptr(s), len(s), _ptr(ds)), "update")
    return s, ds


@dataclass
class CVTResult:
    cell: np.ndarray       # uint32[nz, ny, nx]
    sites: np.ndarray      # uint32[S]
    site_comp: np.ndarray  # uint32[S]
    mean_ds: np.ndarray    # float64[iters]


def cvt(comp: np.ndarray, seeds, weights=None, iters: int = 0) -> CVTResult:
    """Algorithm 1 with a fixed number of updates: T x (VT + update) + final VT."""
    c = np.ascontiguousarray(comp, dtype=np.uint32)
    nx, ny, nz = _dims(c.shape)
    sd = np.ascontiguousarray(seeds, dtype=np.uint32)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.uint16)
    cell = np.empty(c.shape, dtype=np.uint32)
    sites = np.empty(len(sd), dtype=np.uint32)
    sc = np.empty(len(sd), dtype=np.uint32)
    mds = np.zeros(max(iters, 0), dtype=np.float64)
    _check(_load().oracle_cvt(_ptr(c), nx, ny, nz, _ptr(sd), len(sd), _ptr(w), int(iters),
                              _ptr(cell), _ptr(sites), _ptr(sc), _ptr(mds) if iters > 0 else None), "cvt")
    return CVTResult(cell, sites, sc, mds)


@dataclass
class Stats:
    n: np.ndarray      # uint64[U]
    mean: np.ndarray   # float64[U, m]
    m2: np.ndarray     # float64[U, m]   (population variance = m2 / n)
    vmin: np.ndarray   # float32[U, m]
    vmax: np.ndarray   # float32[U, m]
    hist: np.ndarray | None  # uint32[U, m, B]
    cov: np.ndarray | None   # float64[U, m(m+1)/2]  co-moments, packed upper triangle

    @property
    def var(self):
        with np.errstate(invalid="ignore", divide="ignore"):
            return np.where(self.n[:, None] > 0, self.m2 / np.maximum(self.n, 1)[:, None], 0.0)


def stats(unit: np.ndarray, n_units: int, variables: np.ndarray, edges=None, cov: bool = False) -> Stats:
    """Direct two-pass FP64 statistics of each unit (Sec. 3.3 "Aggregation").

    ``unit`` holds a unit id per voxel (NONE_ID = skip); ``variables`` is
    [m, ...] with the spatial shape of ``unit``; ``edges`` is [m, B+1]."""
    u = np.ascontiguousarray(unit, dtype=np.uint32).reshape(-1)
    m = variables.shape[0]
    x = np.ascontiguousarray(variables, dtype=np.float32).reshape(m, -1)
    n = u.size
    e = None if edges is None else np.ascontiguousarray(edges, dtype=np.float32)
    nb = 0 if e is None else e.shape[1] - 1
    U = int(n_units)
    cnt = np.empty(U, dtype=np.uint64)
    mean = np.empty((U, m), dtype=np.float64)
    m2 = np.empty((U, m), dtype=np.float64)
    vmin = np.empty((U, m), dtype=np.float32)
    vmax = np.empty((U, m), dtype=np.float32)
    hist = np.empty((U, m, nb), dtype=np.uint32) if e is not None else None
    P = m * (m + 1) // 2
    cv = np.empty((U, P), dtype=np.float64) if cov else None
    _check(_load().oracle_stats(_ptr(u), n, U, _ptr(x), m, _ptr(e), nb, _ptr(cnt), _ptr(mean), _ptr(m2),
                                _ptr(vmin), _ptr(vmax), _ptr(hist), _ptr(cv)), "stats")
    return Stats(cnt, mean, m2, vmin, vmax, hist, cv)


def chan_merge(n_a, mean_a, m2_a, cov_a, n_b, mean_b, m2_b, cov_b):
    """Pairwise merge of two (n, mean, M2, co-moment) summaries (Chan et al.).

    n = n_a + n_b, delta = mean_b - mean_a, mean = mean_a + delta n_b / n,
    M2 = M2_a + M2_b + delta^2 n_a n_b / n, C_jk = C_a + C_b + delta_j delta_k n_a n_b / n."""
    n = n_a + n_b
    if n == 0:
        return 0, np.zeros_like(mean_a), np.zeros_like(m2_a), None if cov_a is None else np.zeros_like(cov_a)
    if n_a == 0:
        return n_b, mean_b.copy(), m2_b.copy(), None if cov_b is None else cov_b.copy()
    if n_b == 0:
        return n_a, mean_a.copy(), m2_a.copy(), None if cov_a is None else cov_a.copy()
    delta = mean_b - mean_a
    f = float(n_a) * float(n_b) / float(n)
    mean = mean_a + delta * (float(n_b) / float(n))
    m2 = m2_a + m2_b + delta * delta * f
    cv = None
    if cov_a is not None:
        m = len(mean_a)
        dd = np.concatenate([delta[j] * delta[j:] for j in range(m)])
        cv = cov_a + cov_b + dd * f
    return n, mean, m2, cv


@dataclass
class Layout:
    perm: np.ndarray        # uint32[n_placed] voxel linear indices in layout order
    site_order: np.ndarray  # uint32[S] site of the k-th cell
    cell_off: np.ndarray    # uint32[S + 1]
    comp_off: np.ndarray    # uint32[n_comp + 1]
    band_off: np.ndarray    # uint32[n_bands + 1]


def layout(cell: np.ndarray, site_comp, comp_band, n_comp: int, n_bands: int) -> Layout:
    """Structured hierarchical layout (Sec. 3.2.4, Fig. 5).

    Cells are ordered by (component, site id) -- components being numbered
    band-major, this is also band-major -- and the voxels of a cell by linear
    index.  Voxels whose label is not a site id are left out.  A site whose
    component is >= n_comp sorts after every component."""
    c = np.asarray(cell, dtype=np.uint32).ravel()
    sc = np.minimum(np.asarray(site_comp, dtype=np.uint64), n_comp).astype(np.int64)
    S = len(sc)
    order = np.argsort(sc, kind="stable").astype(np.uint32)      # sites by (component, id)
    rank = np.empty(S, dtype=np.int64)
    rank[order] = np.arange(S)
    placed = np.flatnonzero(c < S)
    key = rank[c[placed]]
    perm = placed[np.argsort(key, kind="stable")].astype(np.uint32)  # by cell rank, then index
    per_cell = np.bincount(key, minlength=S)
    cell_off = np.concatenate([[0], np.cumsum(per_cell)]).astype(np.uint32)
    first_rank = np.concatenate([[0], np.cumsum(np.bincount(sc, minlength=n_comp + 1))])[: n_comp + 1]
    comp_off = cell_off[first_rank].astype(np.uint32)
    cb = np.asarray(comp_band, dtype=np.int64)
    first_comp = np.searchsorted(cb, np.arange(n_bands + 1), side="left")
    band_off = comp_off[first_comp].astype(np.uint32)
    return Layout(perm, order, cell_off, comp_off, band_off)


def extract(variables: np.ndarray, perm) -> np.ndarray:
    """out[j][k] = variables[j].flat[perm[k]]."""
    x = np.asarray(variables)
    return x.reshape(x.shape[0], -1)[:, np.asarray(perm, dtype=np.int64)]



# --------------------------------------------------------------------------
# Euclidean line-of-sight tessellation and site update (los_oracle.c)
SITE_FLAG = 0x80000000


def supercover(a, b) -> np.ndarray:
    """Voxels whose closed unit cube meets the segment between the centres
    of voxels a and b, as int32[k, 3] (x, y, z), a first."""
    A = np.ascontiguousarray(a, dtype=np.int32)
    B = np.ascontiguousarray(b, dtype=np.int32)
    cap = int(np.abs(B.astype(np.int64) - A).sum()) * 7 + 2
    out = np.empty((cap, 3), dtype=np.int32)
    k = _load().oracle_supercover(_ptr(A), _ptr(B), _ptr(out), cap)
    if k < 0:
        raise OracleError(ELIMIT, "supercover")
    return out[:k].copy()


@dataclass
class LosVT:
    dist: np.ndarray   # float64[nz, ny, nx]  path length (+inf: no path)
    src: np.ndarray    # uint32[nz, ny, nx]   voxel source, SITE_FLAG | s, or NONE
    phi: np.ndarray    # uint32[nz, ny, nx]   line-of-sight voxel of the path
    cell: np.ndarray   # uint32[nz, ny, nx]   site of phi
    sweeps: tuple      # sweeps run by stage 1 and stage 2


def los_vt(comp: np.ndarray, site_q, anchor) -> LosVT:
    """Restricted Voronoi regions with Euclidean line-of-sight paths (Eq. 1,
    Sec. 3.2.2).  site_q int32[S, 3] in 1/256 voxel, anchor uint32[S]."""
    c = np.ascontiguousarray(comp, dtype=np.uint32)
    nx, ny, nz = _dims(c.shape)
    q = np.ascontiguousarray(site_q, dtype=np.int32).reshape(-1, 3)
    a = np.ascontiguousarray(anchor, dtype=np.uint32)
    dist = np.empty(c.shape, dtype=np.float64)
    src = np.empty(c.shape, dtype=np.uint32)
    phi = np.empty(c.shape, dtype=np.uint32)
    cell = np.empty(c.shape, dtype=np.uint32)
    sw = np.zeros(2, dtype=np.int32)
    _check(_load().oracle_los_vt(_ptr(c), nx, ny, nz, _ptr(q), _ptr(a), len(a), _ptr(dist), _ptr(src),
                                 _ptr(phi), _ptr(cell), _ptr(sw)), "los_vt")
    return LosVT(dist, src, phi, cell, (int(sw[0]), int(sw[1])))


def los_update(comp: np.ndarray, cell: np.ndarray, phi: np.ndarray, site_q, anchor, weights=None):
    """Eq. 2 target with masses carried to line-of-sight voxels, then the
    ray-clamped move (Sec. 3.2.3).  Returns (site_q, anchor, target_q);
    target_q rows of a zero-mass cell are INT32_MIN."""
    c = np.ascontiguousarray(comp, dtype=np.uint32)
    nx, ny, nz = _dims(c.shape)
    q = np.array(site_q, dtype=np.int32, copy=True).reshape(-1, 3)
    a = np.array(anchor, dtype=np.uint32, copy=True)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.uint16)
    t = np.empty_like(q)
    _check(_load().oracle_los_update(_ptr(c), nx, ny, nz, _ptr(w), _ptr(np.ascontiguousarray(cell, dtype=np.uint32)),
                                     _ptr(np.ascontiguousarray(phi, dtype=np.uint32)), len(a), _ptr(q), _ptr(a),
                                     _ptr(t)), "los_update")
    return q, a, t


def los_clamp(comp: np.ndarray, x_q, anchor: int, target_q):
    """The ray-clamped move of one site from x_q (Q8, inside the closed cube
    of voxel `anchor`) towards target_q.  Returns (new x_q, new anchor)."""
    c = np.ascontiguousarray(comp, dtype=np.uint32)
    nx, ny, nz = _dims(c.shape)
    X = np.array(x_q, dtype=np.int32).reshape(3).copy()
    A = np.array([anchor], dtype=np.uint32)
    T = np.array(target_q, dtype=np.int32).reshape(3).copy()
    _check(_load().oracle_los_clamp(_ptr(c), nx, ny, nz, _ptr(X), _ptr(A), _ptr(T)), "los_clamp")
    return X, int(A[0])


@dataclass
class LosCVT:
    site_q: np.ndarray  # int32[S, 3]
    anchor: np.ndarray  # uint32[S]
    dist: np.ndarray
    src: np.ndarray
    phi: np.ndarray
    cell: np.ndarray


def los_cvt(comp: np.ndarray, seeds, weights=None, iters: int = 0) -> LosCVT:
    """Lloyd loop with the line-of-sight tessellation: T x (VT + update) and a
    final VT; sites start at the centres of the seed voxels."""
    c = np.ascontiguousarray(comp, dtype=np.uint32)
    nx, ny, nz = _dims(c.shape)
    sd = np.ascontiguousarray(seeds, dtype=np.uint32)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.uint16)
    q = np.empty((len(sd), 3), dtype=np.int32)
    a = np.empty(len(sd), dtype=np.uint32)
    dist = np.empty(c.shape, dtype=np.float64)
    src = np.empty(c.shape, dtype=np.uint32)
    phi = np.empty(c.shape, dtype=np.uint32)
    cell = np.empty(c.shape, dtype=np.uint32)
    _check(_load().oracle_los_cvt(_ptr(c), nx, ny, nz, _ptr(sd), len(sd), _ptr(w), int(iters), _ptr(q), _ptr(a),
                                  _ptr(dist), _ptr(src), _ptr(phi), _ptr(cell)), "los_cvt")
    return LosCVT(q, a, dist, src, phi, cell)

from .seeding import philox4x32, seed_stratified  # noqa: E402,F401
from .moments import Moments, comoments, tuples  # noqa: E402,F401
