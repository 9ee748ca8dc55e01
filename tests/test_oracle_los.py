"""Pins of the line-of-sight oracle (Euclidean paths of Sec. 3.2.2, the Eq. 2
site update and the ray-clamped move of Sec. 3.2.3) against facts fixed
outside it:

* the supercover walk against a brute-force test of every voxel cube against
  the segment in exact rational arithmetic;
* the clamped move against the first touch of an outside cube found by brute
  force in exact rationals;
* on a convex box every voxel sees its site, so the lengths are the
  Euclidean distances (closed form) and, with two sites, the cells are the two
  sides of the bisector;
* on non-convex domains every length lies between the shortest path in the
  visibility graph of voxel centres (a lower bound: every path the method
  builds is such a path) and the 6-neighbour hop distance plus the anchor
  leg (an upper bound: stage 2 relaxes along face neighbours);
* on a convex box the Eq. 2 target is the plain weighted centroid, rounded to
  1/256 voxel; elsewhere it equals the centroid of the masses carried along
  each path to its line-of-sight voxel, found by following the paths.
"""
import heapq
import itertools
from fractions import Fraction as F

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")
NONE = oracle.NONE_ID
SITE = oracle.SITE_FLAG


# ---------------------------------------------------------------- supercover
def _brute_cover(a, b):
    a = [F(int(t)) for t in a]
    b = [F(int(t)) for t in b]
    D = [b[i] - a[i] for i in range(3)]
    lo = [int(min(a[i], b[i])) - 1 for i in range(3)]
    hi = [int(max(a[i], b[i])) + 1 for i in range(3)]
    out = set()
    for k in itertools.product(*[range(lo[i], hi[i] + 1) for i in range(3)]):
        t0, t1 = F(0), F(1)
        ok = True
        for i in range(3):
            if D[i] == 0:
                if abs(a[i] - k[i]) > F(1, 2):
                    ok = False
                    break
                continue
            u = (k[i] - F(1, 2) - a[i]) / D[i]
            w = (k[i] + F(1, 2) - a[i]) / D[i]
            t0, t1 = max(t0, min(u, w)), min(t1, max(u, w))
        if ok and t0 <= t1:
            out.add(tuple(k))
    return out


def test_supercover_matches_bruteforce():
    rng = np.random.default_rng(7)
    pairs = [((0, 0, 0), (2, 2, 2)), ((0, 0, 0), (3, 1, 0)), ((1, 1, 1), (1, 1, 5)), ((0, 0, 0), (0, 0, 0)),
             ((0, 0, 0), (4, 2, 0)), ((0, 0, 0), (2, 4, 6)), ((5, 0, 3), (0, 5, 0))]
    pairs += [(tuple(rng.integers(-4, 5, 3)), tuple(rng.integers(-4, 5, 3))) for _ in range(150)]
    for a, b in pairs:
        got = oracle.supercover(a, b)
        s = {tuple(int(t) for t in r) for r in got}
        assert len(s) == len(got), (a, b)
        assert tuple(got[0]) == tuple(a)
        assert s == _brute_cover(a, b), (a, b)
        back = {tuple(int(t) for t in r) for r in oracle.supercover(b, a)}
        assert back == s


# ------------------------------------------------------------------- clamping
def _brute_clamp(comp, X, A, T):
    """First t in [0, 1) at which the segment touches the closed cube of a
    voxel outside the component, among the cubes the walk can move into: on
    each axis the segment moves along, the cube must not lie behind the
    anchor's slab; on an axis it does not move along, the cube must be in the
    anchor's slab (faces the segment starts on or slides along do not stop
    it).  Exact rationals over every voxel near the segment."""
    nz, ny, nx = comp.shape
    Ac = (A % nx, (A // nx) % ny, A // (nx * ny))
    P = [F(int(x), 256) for x in X]
    Q = [F(int(t), 256) for t in T]
    D = [Q[i] - P[i] for i in range(3)]
    if all(d == 0 for d in D):
        return list(X), A
    c = comp.ravel()[A]
    lo = [int(min(P[i], Q[i])) - 2 for i in range(3)]
    hi = [int(max(P[i], Q[i])) + 2 for i in range(3)]
    best = None
    for k in itertools.product(*[range(lo[i], hi[i] + 1) for i in range(3)]):
        x, y, z = k
        inside = 0 <= x < nx and 0 <= y < ny and 0 <= z < nz
        if inside and comp[z, y, x] == c:
            continue
        t0, t1 = F(0), F(1)
        ok = True
        for i in range(3):
            if D[i] == 0:
                if k[i] != Ac[i]:
                    ok = False
                    break
                continue
            u = (k[i] - F(1, 2) - P[i]) / D[i]
            w = (k[i] + F(1, 2) - P[i]) / D[i]
            if (k[i] - Ac[i]) * (1 if D[i] > 0 else -1) < 0:  # behind the anchor
                ok = False
                break
            t0, t1 = max(t0, min(u, w)), min(t1, max(u, w))
        if ok and t0 <= t1 and t0 < 1 and (best is None or t0 < best):
            best = t0
    if best is None:
        tt, newX = F(1), [int(t) for t in T]
    else:
        tt = best
        newX = [int(X[i]) + int(tt * (int(T[i]) - int(X[i]))) for i in range(3)]
    if tt == 0:
        return newX, A
    eps = F(1, 2 ** 70)
    p = [P[i] + (tt - eps) * D[i] for i in range(3)]
    v = [Ac[i] if D[i] == 0 else int(np.floor(p[i] + F(1, 2))) for i in range(3)]
    return newX, v[0] + nx * (v[1] + ny * v[2])


def test_clamp_matches_bruteforce():
    rng = np.random.default_rng(11)
    for trial in range(120):
        nz = 1 if trial % 3 == 0 else 4
        shape = (nz, 7, 8)
        comp = np.where(rng.random(shape) < 0.25, NONE, 0).astype(np.uint32)
        cand = np.flatnonzero(comp.ravel() == 0)
        if len(cand) == 0:
            continue
        A = int(rng.choice(cand))
        ax, ay, az = A % 8, (A // 8) % 7, A // 56
        off = rng.integers(-128, 129, 3)
        if trial % 4 == 0:
            off = rng.choice([-128, 0, 128], 3)  # on faces, edges and corners
        X = [256 * ax + off[0], 256 * ay + off[1], 256 * az + off[2] if nz > 1 else 0]
        T = [int(rng.integers(-300, 256 * 8 + 300)), int(rng.integers(-300, 256 * 7 + 300)),
             int(rng.integers(-300, 256 * nz + 300)) if nz > 1 else 0]
        if trial % 5 == 0:
            T = [256 * int(rng.integers(0, 8)) + 128, 256 * int(rng.integers(0, 7)), X[2]]
        got_x, got_a = oracle.los_clamp(comp, X, A, T)
        want_x, want_a = _brute_clamp(comp, X, A, T)
        assert list(got_x) == want_x, (trial, X, A, T)
        assert got_a == want_a, (trial, X, A, T)
        # the new position lies in the closed cube of the new anchor, inside C
        q = got_a
        assert comp.ravel()[q] == comp.ravel()[A]
        qc = np.array([q % 8, (q // 8) % 7, q // 56])
        assert np.all(np.abs(256 * qc - np.asarray(got_x)) <= 128)


# -------------------------------------------------------------- convex boxes
def _grid(shape):
    z, y, x = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    return x.astype(np.int64), y.astype(np.int64), z.astype(np.int64)


def test_los_box_one_site_is_euclidean():
    shape = (9, 11, 13)
    comp = np.full(shape, 5, dtype=np.uint32)
    q = np.array([[4 * 256 + 77, 6 * 256 - 100, 3 * 256 + 128]], dtype=np.int32)
    a = np.array([4 + 13 * (6 + 11 * 3)], dtype=np.uint32)
    r = oracle.los_vt(comp, q, a)
    x, y, z = _grid(shape)
    n2 = (256 * x - q[0, 0]) ** 2 + (256 * y - q[0, 1]) ** 2 + (256 * z - q[0, 2]) ** 2
    np.testing.assert_array_equal(r.dist, np.sqrt(n2.astype(np.float64)) / 256.0)
    assert np.all(r.src == SITE)
    np.testing.assert_array_equal(r.phi.ravel(), np.arange(comp.size))
    assert np.all(r.cell == 0)


def test_los_box_two_sites_bisector():
    shape = (7, 12, 10)
    comp = np.zeros(shape, dtype=np.uint32)
    x, y, z = _grid(shape)
    rng = np.random.default_rng(3)
    for trial in range(4):
        vox = rng.choice(comp.size, 2, replace=False)
        q = np.array([[256 * (v % 10), 256 * ((v // 10) % 12), 256 * (v // 120)] for v in vox], dtype=np.int32)
        q[:, :2] += rng.integers(-128, 129, (2, 2)).astype(np.int32)
        r = oracle.los_vt(comp, q, vox.astype(np.uint32))
        n2 = [(256 * x - q[s, 0]) ** 2 + (256 * y - q[s, 1]) ** 2 + (256 * z - q[s, 2]) ** 2 for s in range(2)]
        want = np.where(n2[1] < n2[0], 1, 0)
        np.testing.assert_array_equal(r.cell, want)
        np.testing.assert_array_equal(r.dist, np.sqrt(np.minimum(*n2).astype(np.float64)) / 256.0)
        assert np.all(r.src & SITE)


def test_los_update_box_is_plain_centroid():
    shape = (6, 9, 11)
    comp = np.zeros(shape, dtype=np.uint32)
    rng = np.random.default_rng(5)
    w = rng.integers(0, 1000, shape).astype(np.uint16)
    vox = rng.choice(comp.size, 3, replace=False)
    q = np.array([[256 * (v % 11), 256 * ((v // 11) % 9), 256 * (v // 99)] for v in vox], dtype=np.int32)
    r = oracle.los_vt(comp, q, vox.astype(np.uint32))
    nq, na, tq = oracle.los_update(comp, r.cell, r.phi, q, vox.astype(np.uint32), w)
    x, y, z = _grid(shape)
    for s in range(3):
        m = r.cell == s
        M = int(w[m].astype(np.int64).sum())
        for i, coord in enumerate((x, y, z)):
            S = int((w[m].astype(np.int64) * coord[m]).sum())
            want = int(np.floor(F(256 * S, M) + F(1, 2)))
            assert tq[s, i] == want
        # a convex box never blocks: the site reaches its target
        np.testing.assert_array_equal(nq[s], tq[s])
        ac = np.array([na[s] % 11, (na[s] // 11) % 9, na[s] // 99])
        assert np.all(np.abs(256 * ac - nq[s]) <= 128)


# ---------------------------------------------------------- non-convex bounds
def _domain(seed, shape=(3, 12, 14)):
    rng = np.random.default_rng(seed)
    free = rng.random(shape) > 0.22
    # keep the largest 6-connected free component as C
    lab = np.full(shape, -1)
    best, bsz = -1, 0
    k = 0
    for start in zip(*np.nonzero(free)):
        if lab[start] >= 0:
            continue
        st, size = [start], 0
        lab[start] = k
        while st:
            p = st.pop()
            size += 1
            for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                q = (p[0] + d[0], p[1] + d[1], p[2] + d[2])
                if all(0 <= q[i] < shape[i] for i in range(3)) and free[q] and lab[q] < 0:
                    lab[q] = k
                    st.append(q)
        if size > bsz:
            best, bsz = k, size
        k += 1
    return np.where(lab == best, 0, NONE).astype(np.uint32)


def _visible(comp, u, v):
    nz, ny, nx = comp.shape
    c = comp.ravel()[u]
    a = (u % nx, (u // nx) % ny, u // (nx * ny))
    b = (v % nx, (v // nx) % ny, v // (nx * ny))
    for x, y, z in oracle.supercover(a, b):
        if not (0 <= x < nx and 0 <= y < ny and 0 <= z < nz) or comp[z, y, x] != c:
            return False
    return True


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_los_lengths_between_visibility_graph_and_hops(seed):
    comp = _domain(seed)
    nz, ny, nx = comp.shape
    flat = comp.ravel()
    cells = np.flatnonzero(flat == 0)
    rng = np.random.default_rng(seed)
    anchors = rng.choice(cells, 3, replace=False).astype(np.uint32)
    q = np.array([[256 * (v % nx), 256 * ((v // nx) % ny), 256 * (v // (nx * ny))] for v in anchors],
                 dtype=np.int32)
    r = oracle.los_vt(comp, q, anchors)
    d = r.dist.ravel()
    assert np.all(np.isfinite(d[cells])) and np.all(np.isinf(d[flat != 0]))

    coord = lambda v: np.array([v % nx, (v // nx) % ny, v // (nx * ny)], dtype=np.int64)
    # lower bound: Dijkstra over voxel centres joined when mutually visible,
    # each site joined to the voxels that see its anchor
    vis = {}
    for u in cells:
        for v in cells:
            if u < v and _visible(comp, u, v):
                vis.setdefault(u, []).append(v)
                vis.setdefault(v, []).append(u)
    low = np.full(flat.size, np.inf)
    heap = []
    for s, a in enumerate(anchors):
        for v in [int(a)] + vis.get(int(a), []):
            dv = np.sqrt(float(((256 * coord(v) - q[s]) ** 2).sum())) / 256.0
            if dv < low[v]:
                low[v] = dv
                heapq.heappush(heap, (dv, v))
    while heap:
        dv, v = heapq.heappop(heap)
        if dv > low[v]:
            continue
        for u in vis.get(v, []):
            du = dv + np.sqrt(float(((coord(u) - coord(v)) ** 2).sum()))
            if du < low[u]:
                low[u] = du
                heapq.heappush(heap, (du, u))
    assert np.all(d[cells] >= low[cells] * (1 - 1e-12))

    # upper bound: hops along face neighbours from an anchor, plus its leg
    up = np.full(flat.size, np.inf)
    for s, a in enumerate(anchors):
        hop = np.full(flat.size, -1)
        hop[a] = 0
        fr = [int(a)]
        while fr:
            nxt = []
            for v in fr:
                x, y, z = coord(v)
                for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    X, Y, Z = x + dx, y + dy, z + dz
                    if 0 <= X < nx and 0 <= Y < ny and 0 <= Z < nz:
                        u = X + nx * (Y + ny * Z)
                        if flat[u] == 0 and hop[u] < 0:
                            hop[u] = hop[v] + 1
                            nxt.append(u)
            fr = nxt
        leg = np.sqrt(float(((256 * coord(int(a)) - q[s]) ** 2).sum())) / 256.0
        up = np.minimum(up, np.where(hop >= 0, hop + leg, np.inf))
    assert np.all(d[cells] <= up[cells] * (1 + 1e-9))

    # every recorded path is a chain of clear segments ending at a site
    src = r.src.ravel()
    for v in cells:
        u = int(src[v])
        if u & SITE:
            s = u & (SITE - 1)
            assert _visible(comp, int(v), int(anchors[s]))
            assert d[v] == np.sqrt(float(((256 * coord(v) - q[s]) ** 2).sum())) / 256.0
        else:
            assert _visible(comp, int(v), u)
            leg = np.sqrt(float(((coord(v) - coord(u)) ** 2).sum()))
            assert abs(d[v] - (leg + d[u])) <= 1e-9 * d[v]
            assert d[u] < d[v]
    # the cell of v is the site of its line-of-sight voxel phi(v)
    phi = r.phi.ravel()
    assert np.all(src[phi[cells]] & SITE)
    np.testing.assert_array_equal(r.cell.ravel()[cells], src[phi[cells]] & (SITE - 1))


def test_los_update_carries_mass_along_paths():
    comp = _domain(4, shape=(2, 13, 15))
    nz, ny, nx = comp.shape
    flat = comp.ravel()
    cells = np.flatnonzero(flat == 0)
    rng = np.random.default_rng(4)
    anchors = rng.choice(cells, 4, replace=False).astype(np.uint32)
    q = np.array([[256 * (v % nx), 256 * ((v // nx) % ny), 256 * (v // (nx * ny))] for v in anchors],
                 dtype=np.int32)
    w = rng.integers(1, 50, comp.shape).astype(np.uint16)
    r = oracle.los_vt(comp, q, anchors)
    src = r.src.ravel()
    assert np.any((src[cells] & SITE) == 0), "the domain should have voxels out of sight"
    M = np.zeros(4, dtype=object)
    S = np.zeros((4, 3), dtype=object)
    for v in cells:
        u = int(v)
        while not (src[u] & SITE):  # follow the path to its line-of-sight voxel
            u = int(src[u])
        s = int(src[u] & (SITE - 1))
        m = int(w.ravel()[v])
        M[s] += m
        S[s] += m * np.array([u % nx, (u // nx) % ny, u // (nx * ny)], dtype=object)
    _, _, tq = oracle.los_update(comp, r.cell, r.phi, q, anchors, w)
    for s in range(4):
        if M[s] == 0:
            assert np.all(tq[s] == np.iinfo(np.int32).min)
            continue
        for i in range(3):
            assert tq[s, i] == int(np.floor(F(256 * int(S[s, i]), int(M[s])) + F(1, 2)))
    # mass conservation: every voxel's mass lands on exactly one site
    assert sum(M) == int(w.ravel()[cells].astype(np.int64).sum())


def test_los_cvt_keeps_sites_inside_their_component():
    comp = _domain(6, shape=(3, 14, 16))
    nz, ny, nx = comp.shape
    cells = np.flatnonzero(comp.ravel() == 0)
    rng = np.random.default_rng(6)
    seeds = rng.choice(cells, 5, replace=False).astype(np.uint32)
    res = oracle.los_cvt(comp, seeds, None, iters=4)
    for s in range(5):
        a = int(res.anchor[s])
        assert comp.ravel()[a] == 0
        ac = np.array([a % nx, (a // nx) % ny, a // (nx * ny)])
        assert np.all(np.abs(256 * ac - res.site_q[s]) <= 128)
    assert np.all(res.cell.ravel()[cells] < 5)
