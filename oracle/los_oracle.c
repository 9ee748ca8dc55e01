/*
 * Plain CPU oracle for the Euclidean, line-of-sight form of the restricted
 * Voronoi tessellation and its site update (Sec. 3.1 "Centroids or Centers of
 * Mass" with Eq. 2; Sec. 3.2.2 "Discrete Restricted Geodesic Voronoi
 * Tessellation"; Sec. 3.2.3 "Geodesically Weighted Voronoi Site Update").
 *
 * TEST INFRASTRUCTURE ONLY.  Built into the same oracle library as
 * lsrvt_oracle.c; the GPU library never links, calls or includes it.
 *
 * Readings (the paper leaves these open):
 *  - A voxel is a closed unit cube centred on its integer coordinates.  The
 *    segment between two points is clear when every voxel whose closed cube
 *    meets the closed segment belongs to the component (the "supercover" of
 *    the segment; grazing an edge or a corner of an outside voxel blocks).
 *  - A site is a continuous point X_s, kept in fixed point with 8 fraction
 *    bits (Q8: X = 256 x), plus an anchor voxel: the voxel the site sits in,
 *    the voxel where its region starts growing.  Line of sight between a voxel
 *    v and the site is tested on the segment from v to the anchor's centre;
 *    the length of that leg is |x_v - X_s|.
 *  - Path lengths are float64: sqrt of an exact integer squared length
 *    (voxel to voxel), or sqrt of the exact Q8 squared length divided by 256
 *    (voxel to site), plus the length stored at the source.
 *  - src(v) is either another voxel u (the path continues at u) or the site
 *    itself, coded SITE_FLAG | s; the latter are exactly the line-of-sight
 *    voxels, so los(v) = (src(v) has SITE_FLAG).
 *  - Rounding makes a path through a voxel on the straight line to the site
 *    as long as the straight line, or an ulp shorter.  So a voxel takes a
 *    new path only when the shortest valid candidate d_min is shorter than
 *    the held length by a relative 2^-40, and then takes, among the valid
 *    candidates no longer than d_min (1 + 2^-40), the site itself first
 *    (lowest id), else the lowest voxel index.  The anchor step compares
 *    (length, site id) exactly.
 *  - The relaxation is synchronous (Jacobi): every sweep reads the state of
 *    the previous sweep only, as the delayed update of Sec. 3.2.2 requires.
 *    A voxel v in the component of an active neighbour w considers
 *      (a) the path through src(w): to the site if src(w) is a site (the ray
 *          to the anchor must be clear), else |x_v - x_u| + d[u] for
 *          u = src(w) != v (the ray v -> u must be clear);
 *      (b) the path through w: d[w] + 1 (face neighbours are always clear);
 *      (c) its own path re-measured, |x_v - x_u| + d[u] for its current
 *          voxel source u, so that a stored length tracks a source that got
 *          shorter (no ray: it was clear when u was taken).
 *    Stage 1 (only the sites are path nodes) allows (a) through sites only;
 *    it ends when a sweep changes nothing.  Stage 2 (every voxel a node)
 *    allows all three and also ends when a sweep changes nothing.
 *  - phi(v) = v if los(v) else phi(src(v)) (Eq. 2); the cell of v is the site
 *    of phi(v).
 *  - Site update (Eq. 2): M = sum m_v and S = sum m_v x_{phi(v)} over the cell
 *    in exact integers; the target X_c = round-half-up(256 S / M) in Q8.  The
 *    site then walks the segment X_s -> X_c voxel by voxel from its anchor and
 *    stops at the first parameter t < 1 at which the segment touches the
 *    closed cube of a voxel outside the component (or the volume), counting
 *    only the cubes the walk can move into: none behind the anchor on an axis
 *    the segment moves along, none beside it on an axis it does not move
 *    along (so a site on a boundary face can leave it, or slide along it);
 *    the new
 *    position is X_s + trunc(t (X_c - X_s)) per axis and the new anchor is the
 *    voxel the walk stopped in.  If nothing is touched before t = 1 the site
 *    reaches X_c.  A cell of zero mass keeps its site.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LOS_OK 0
#define LOS_EINVAL 1
#define LOS_ENOMEM 3
#define LOS_ELIMIT 4

#define LOS_NONE 0xFFFFFFFFu
#define SITE_FLAG 0x80000000u
#define LOS_MAX_SWEEPS 100000
/* A path replaces the held one only when shorter by a relative 2^-40, far
 * above the rounding of a sum of path legs; paths within 2^-40 of the
 * shortest count as equally long.                                           */
#define LOS_SHORTER (1.0 - 0x1p-40)
#define LOS_NEAR (1.0 + 0x1p-40)

typedef struct { int64_t x, y, z; } ivec;

static ivec coords(int64_t v, int32_t nx, int32_t ny) {
    ivec c;
    c.x = v % nx;
    c.y = (v / nx) % ny;
    c.z = v / ((int64_t)nx * ny);
    return c;
}

static int inside(ivec c, int32_t nx, int32_t ny, int32_t nz) {
    return c.x >= 0 && c.y >= 0 && c.z >= 0 && c.x < nx && c.y < ny && c.z < nz;
}

static int64_t lin(ivec c, int32_t nx, int32_t ny) { return c.x + (int64_t)nx * (c.y + (int64_t)ny * c.z); }

/* Supercover of the segment between the centres of voxels a and b.  With
 * L_i = |b_i - a_i|, the segment crosses the planes between voxels of axis i
 * at t = (2k + 1) / (2 L_i), k = 0..L_i-1.  Crossings are taken in order of t
 * (compared exactly by cross-multiplication); when several axes cross at the
 * same t the segment passes through an edge or a corner and every voxel that
 * combines the old and new index of those axes is touched.  visit() is called
 * on each voxel of the cover except a itself; it returns 0 to stop the walk.
 * Returns 1 if the walk finished, 0 if visit() stopped it.                   */
typedef int (*visit_fn)(ivec c, void *ctx);

static int supercover_walk(ivec a, ivec b, visit_fn visit, void *ctx) {
    int64_t L[3] = {llabs(b.x - a.x), llabs(b.y - a.y), llabs(b.z - a.z)};
    int64_t s[3] = {b.x > a.x ? 1 : -1, b.y > a.y ? 1 : -1, b.z > a.z ? 1 : -1};
    int64_t m[3] = {0, 0, 0};
    int64_t cur[3] = {a.x, a.y, a.z};
    for (;;) {
        int best = -1;
        for (int i = 0; i < 3; ++i) {
            if (m[i] >= L[i]) continue;
            if (best < 0 || (2 * m[i] + 1) * L[best] < (2 * m[best] + 1) * L[i]) best = i;
        }
        if (best < 0) return 1;
        int tied[3], nt = 0;
        for (int i = 0; i < 3; ++i)
            if (m[i] < L[i] && (2 * m[i] + 1) * L[best] == (2 * m[best] + 1) * L[i]) tied[nt++] = i;
        for (int mask = 1; mask < (1 << nt); ++mask) {
            int64_t c[3] = {cur[0], cur[1], cur[2]};
            for (int j = 0; j < nt; ++j)
                if (mask & (1 << j)) c[tied[j]] += s[tied[j]];
            ivec cv = {c[0], c[1], c[2]};
            if (!visit(cv, ctx)) return 0;
        }
        for (int j = 0; j < nt; ++j) {
            cur[tied[j]] += s[tied[j]];
            m[tied[j]] += 1;
        }
    }
}

typedef struct {
    const uint32_t *comp;
    int32_t nx, ny, nz;
    uint32_t c;
} clear_ctx;

static int clear_visit(ivec c, void *p) {
    clear_ctx *k = (clear_ctx *)p;
    if (!inside(c, k->nx, k->ny, k->nz)) return 0;
    return k->comp[lin(c, k->nx, k->ny)] == k->c;
}

static int ray_clear(const uint32_t *comp, int32_t nx, int32_t ny, int32_t nz, int64_t v, int64_t u) {
    clear_ctx k = {comp, nx, ny, nz, comp[v]};
    return supercover_walk(coords(v, nx, ny), coords(u, nx, ny), clear_visit, &k);
}

typedef struct {
    int32_t *out;
    int64_t cap, n;
} list_ctx;

static int list_visit(ivec c, void *p) {
    list_ctx *k = (list_ctx *)p;
    if (k->n >= k->cap) return 0;
    k->out[3 * k->n + 0] = (int32_t)c.x;
    k->out[3 * k->n + 1] = (int32_t)c.y;
    k->out[3 * k->n + 2] = (int32_t)c.z;
    k->n += 1;
    return 1;
}

/* The supercover of the segment a -> b as a list of (x, y, z), a first;
 * returns the count, or -1 when cap is too small.                            */
int64_t oracle_supercover(const int32_t *a, const int32_t *b, int32_t *out, int64_t cap) {
    if (cap < 1) return -1;
    out[0] = a[0]; out[1] = a[1]; out[2] = a[2];
    list_ctx k = {out + 3, cap - 1, 0};
    ivec A = {a[0], a[1], a[2]}, B = {b[0], b[1], b[2]};
    if (!supercover_walk(A, B, list_visit, &k)) return -1;
    return k.n + 1;
}

static double dist_vox(ivec a, ivec b) {
    int64_t dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    return sqrt((double)(dx * dx + dy * dy + dz * dz));
}

static double dist_site(ivec a, const int32_t *q) {
    int64_t dx = 256 * a.x - q[0], dy = 256 * a.y - q[1], dz = 256 * a.z - q[2];
    return sqrt((double)(dx * dx + dy * dy + dz * dz)) / 256.0;
}

/* Preference among paths of (nearly) equal length: the site itself first
 * (ids ascending), then voxel sources (indices ascending).                  */
static uint32_t pref(uint32_t code) { return code ^ SITE_FLAG; }

/* One synchronous sweep: new state from old for every component voxel.
 * Returns the number of voxels that changed.                                 */
static int64_t los_sweep(const uint32_t *comp, int32_t nx, int32_t ny, int32_t nz, int64_t n,
                         const int32_t *site_q, const uint32_t *anchor, int stage,
                         const double *d_old, const uint32_t *s_old, double *d_new, uint32_t *s_new) {
    int64_t changed = 0;
    for (int64_t v = 0; v < n; ++v) {
        d_new[v] = d_old[v];
        s_new[v] = s_old[v];
        uint32_t c = comp[v];
        if (c == LOS_NONE) continue;
        ivec pv = coords(v, nx, ny);
        /* candidate list: (length, code, ray target voxel or -1) */
        double cd[13];
        uint32_t cc[13];
        int64_t ray[13];
        int nc = 0;
        if (stage == 2 && s_old[v] != LOS_NONE && !(s_old[v] & SITE_FLAG)) {
            int64_t u = s_old[v];
            cd[nc] = dist_vox(pv, coords(u, nx, ny)) + d_old[u];
            cc[nc] = (uint32_t)u;
            ray[nc++] = -1;
        }
        int64_t nb[6];
        int k = 0;
        if (pv.x > 0) nb[k++] = v - 1;
        if (pv.x < nx - 1) nb[k++] = v + 1;
        if (pv.y > 0) nb[k++] = v - nx;
        if (pv.y < ny - 1) nb[k++] = v + nx;
        if (pv.z > 0) nb[k++] = v - (int64_t)nx * ny;
        if (pv.z < nz - 1) nb[k++] = v + (int64_t)nx * ny;
        for (int i = 0; i < k; ++i) {
            int64_t w = nb[i];
            if (comp[w] != c || s_old[w] == LOS_NONE) continue;
            uint32_t u = s_old[w];
            if (u & SITE_FLAG) {
                uint32_t s = u & ~SITE_FLAG;
                cd[nc] = dist_site(pv, site_q + 3 * (int64_t)s);
                cc[nc] = u;
                ray[nc++] = anchor[s];
            } else if (stage == 2 && (int64_t)u != v) {
                cd[nc] = dist_vox(pv, coords(u, nx, ny)) + d_old[u];
                cc[nc] = u;
                ray[nc++] = u;
            }
            if (stage == 2) {
                cd[nc] = d_old[w] + 1.0;
                cc[nc] = (uint32_t)w;
                ray[nc++] = -1;
            }
        }
        /* Candidates no shorter than the held path cannot matter; the others
         * are valid when their ray is clear.  The shortest valid length
         * d_min must beat the held one by the relative margin; then the
         * preferred candidate within the margin above d_min is taken.      */
        double dh = d_old[v];
        int valid[13];
        double dmin = INFINITY;
        for (int i = 0; i < nc; ++i) {
            valid[i] = cd[i] < dh && (ray[i] < 0 || ray_clear(comp, nx, ny, nz, v, ray[i]));
            if (valid[i] && cd[i] < dmin) dmin = cd[i];
        }
        if (!(dmin < dh * LOS_SHORTER)) continue;
        double lim = dmin * LOS_NEAR;
        int sel = -1;
        for (int i = 0; i < nc; ++i) {
            if (!valid[i] || cd[i] > lim) continue;
            if (sel < 0 || pref(cc[i]) < pref(cc[sel]) || (cc[i] == cc[sel] && cd[i] < cd[sel])) sel = i;
        }
        d_new[v] = cd[sel];
        s_new[v] = cc[sel];
        ++changed;
    }
    return changed;
}

static int check_sites(const uint32_t *comp, int64_t n, int32_t nx, int32_t ny, int32_t nz,
                       const int32_t *site_q, const uint32_t *anchor, uint32_t n_sites) {
    if (n_sites >= SITE_FLAG - 1) return LOS_ELIMIT;
    for (uint32_t s = 0; s < n_sites; ++s) {
        if ((int64_t)anchor[s] >= n) return LOS_EINVAL;
        if (comp[anchor[s]] == LOS_NONE) return LOS_EINVAL;
        ivec a = coords(anchor[s], nx, ny);
        const int32_t *q = site_q + 3 * (int64_t)s;
        /* the site must lie in the closed cube of its anchor */
        if (llabs(256 * a.x - q[0]) > 128 || llabs(256 * a.y - q[1]) > 128 || llabs(256 * a.z - q[2]) > 128)
            return LOS_EINVAL;
    }
    (void)nz;
    return LOS_OK;
}

static int los_dims(int32_t nx, int32_t ny, int32_t nz, int64_t *n) {
    if (nx <= 0 || ny <= 0 || nz <= 0) return LOS_EINVAL;
    if (nx > 32767 || ny > 32767 || nz > 32767) return LOS_ELIMIT;
    *n = (int64_t)nx * ny * nz;
    if (*n > 2147483647LL) return LOS_ELIMIT;
    return LOS_OK;
}

/* Restricted Voronoi tessellation with Euclidean path lengths and
 * line-of-sight shortcuts (Eq. 1 with the paths of Sec. 3.2.2).
 *   site_q  int32[S][3]  Q8 site positions;  anchor uint32[S] anchor voxels
 *   dist    float64[N]   path length (+inf where no path)
 *   src     uint32[N]    voxel source, SITE_FLAG | s, or LOS_NONE
 *   phi     uint32[N]    the line-of-sight voxel of the path (LOS_NONE)
 *   cell    uint32[N]    the site of phi (LOS_NONE)
 *   sweeps  int32[2]     sweeps run by stage 1 and stage 2 (may be NULL)    */
int oracle_los_vt(const uint32_t *comp, int32_t nx, int32_t ny, int32_t nz,
                  const int32_t *site_q, const uint32_t *anchor, uint32_t n_sites,
                  double *dist, uint32_t *src, uint32_t *phi, uint32_t *cell, int32_t *sweeps) {
    int64_t n;
    int st = los_dims(nx, ny, nz, &n);
    if (st) return st;
    st = check_sites(comp, n, nx, ny, nz, site_q, anchor, n_sites);
    if (st) return st;
    double *d2 = (double *)malloc(sizeof(double) * n);
    uint32_t *s2 = (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!d2 || !s2) { free(d2); free(s2); return LOS_ENOMEM; }
    for (int64_t v = 0; v < n; ++v) { dist[v] = INFINITY; src[v] = LOS_NONE; }
    /* the initial step: each anchor holds its site (the smaller key wins) */
    for (uint32_t s = 0; s < n_sites; ++s) {
        int64_t a = anchor[s];
        double d = dist_site(coords(a, nx, ny), site_q + 3 * (int64_t)s);
        if (d < dist[a] || (d == dist[a] && s < (src[a] & ~SITE_FLAG))) { dist[a] = d; src[a] = SITE_FLAG | s; }
    }
    for (int stage = 1; stage <= 2 && !st; ++stage) {
        int32_t k = 0;
        for (;;) {
            if (k >= LOS_MAX_SWEEPS) { st = LOS_ELIMIT; break; }
            int64_t ch = los_sweep(comp, nx, ny, nz, n, site_q, anchor, stage, dist, src, d2, s2);
            ++k;
            memcpy(dist, d2, sizeof(double) * n);
            memcpy(src, s2, sizeof(uint32_t) * n);
            if (ch == 0) break;
        }
        if (sweeps) sweeps[stage - 1] = k;
    }
    free(d2);
    free(s2);
    if (st) return st;
    /* phi by following each path to its line-of-sight voxel */
    for (int64_t v = 0; v < n; ++v) {
        phi[v] = LOS_NONE;
        cell[v] = LOS_NONE;
        if (src[v] == LOS_NONE) continue;
        int64_t u = v;
        int64_t hops = 0;
        while (!(src[u] & SITE_FLAG)) {
            u = src[u];
            if (++hops > n) return LOS_ELIMIT; /* a cycle: cannot happen */
        }
        phi[v] = (uint32_t)u;
        cell[v] = src[u] & ~SITE_FLAG;
    }
    return LOS_OK;
}

/* The ray-clamped move of one site (Sec. 3.2.3): from X (Q8) in voxel A
 * towards T, stopping where the segment first touches a voxel outside
 * component c.  Event times along axis i are (plane - X_i) / (T_i - X_i) with
 * the planes at 256 k +- 128; they are compared by cross-multiplication.    */
static void clamp_move(const uint32_t *comp, int32_t nx, int32_t ny, int32_t nz, uint32_t c,
                       int32_t *X, uint32_t *A, const int64_t *T) {
    int64_t D[3], num[3], den[3], step[3];
    ivec cur = coords(*A, nx, ny);
    int64_t cv[3] = {cur.x, cur.y, cur.z};
    for (int i = 0; i < 3; ++i) {
        D[i] = T[i] - X[i];
        step[i] = D[i] > 0 ? 1 : -1;
        den[i] = llabs(D[i]);
        /* distance from X to the next plane in the direction of travel */
        int64_t plane = 256 * cv[i] + 128 * step[i];
        num[i] = (plane - X[i]) * step[i];
    }
    if (D[0] == 0 && D[1] == 0 && D[2] == 0) return;
    for (;;) {
        int best = -1;
        for (int i = 0; i < 3; ++i) {
            if (den[i] == 0 || num[i] >= den[i]) continue; /* no crossing before t = 1 */
            if (best < 0 || num[i] * den[best] < num[best] * den[i]) best = i;
        }
        if (best < 0) break;
        int tied[3], nt = 0;
        for (int i = 0; i < 3; ++i)
            if (den[i] != 0 && num[i] < den[i] && num[i] * den[best] == num[best] * den[i]) tied[nt++] = i;
        int blocked = 0;
        for (int mask = 1; mask < (1 << nt) && !blocked; ++mask) {
            ivec q = {cv[0], cv[1], cv[2]};
            int64_t *qa[3] = {&q.x, &q.y, &q.z};
            for (int j = 0; j < nt; ++j)
                if (mask & (1 << j)) *qa[tied[j]] += step[tied[j]];
            if (!inside(q, nx, ny, nz) || comp[lin(q, nx, ny)] != c) blocked = 1;
        }
        if (blocked) {
            int64_t tn = num[best], td = den[best];
            for (int i = 0; i < 3; ++i) X[i] = (int32_t)(X[i] + (tn * D[i]) / td);
            ivec e = {cv[0], cv[1], cv[2]};
            *A = (uint32_t)lin(e, nx, ny);
            return;
        }
        for (int j = 0; j < nt; ++j) {
            cv[tied[j]] += step[tied[j]];
            num[tied[j]] += 256;
        }
    }
    for (int i = 0; i < 3; ++i) X[i] = (int32_t)T[i];
    ivec e = {cv[0], cv[1], cv[2]};
    *A = (uint32_t)lin(e, nx, ny);
}

/* The clamped move alone, for the tests: X (Q8, in/out), anchor A (in/out),
 * target T (Q8), walking through the component of A.                        */
int oracle_los_clamp(const uint32_t *comp, int32_t nx, int32_t ny, int32_t nz, int32_t *X, uint32_t *A,
                     const int32_t *T) {
    int64_t n;
    int st = los_dims(nx, ny, nz, &n);
    if (st) return st;
    if ((int64_t)*A >= n || comp[*A] == LOS_NONE) return LOS_EINVAL;
    int64_t t[3] = {T[0], T[1], T[2]};
    clamp_move(comp, nx, ny, nz, comp[*A], X, A, t);
    return LOS_OK;
}

/* Geodesically weighted site update (Eq. 2, Sec. 3.2.3).  M, S in uint64
 * (weights are uint16 and coordinates below 2^15, so S < 2^62); the target
 * is round-half-up(256 S / M) per axis, done as 256 q + floor((512 r + M) /
 * (2 M)) with S = q M + r.  target_q (may be NULL) receives the targets
 * (INT32_MIN for a cell of zero mass).  weights NULL means m_v = 1.         */
int oracle_los_update(const uint32_t *comp, int32_t nx, int32_t ny, int32_t nz, const uint16_t *weights,
                      const uint32_t *cell, const uint32_t *phi, uint32_t n_sites,
                      int32_t *site_q, uint32_t *anchor, int32_t *target_q) {
    int64_t n;
    int st = los_dims(nx, ny, nz, &n);
    if (st) return st;
    uint64_t *acc = (uint64_t *)calloc(4 * (size_t)(n_sites ? n_sites : 1), sizeof(uint64_t));
    if (!acc) return LOS_ENOMEM;
    for (int64_t v = 0; v < n; ++v) {
        uint32_t s = cell[v];
        if (s == LOS_NONE) continue;
        if (s >= n_sites) { free(acc); return LOS_EINVAL; }
        uint64_t m = weights ? weights[v] : 1;
        ivec p = coords(phi[v], nx, ny);
        acc[4 * (size_t)s + 0] += m;
        acc[4 * (size_t)s + 1] += m * (uint64_t)p.x;
        acc[4 * (size_t)s + 2] += m * (uint64_t)p.y;
        acc[4 * (size_t)s + 3] += m * (uint64_t)p.z;
    }
    for (uint32_t s = 0; s < n_sites; ++s) {
        uint64_t M = acc[4 * (size_t)s];
        if (M == 0) {
            if (target_q) target_q[3 * (size_t)s] = target_q[3 * (size_t)s + 1] = target_q[3 * (size_t)s + 2] = INT32_MIN;
            continue;
        }
        int64_t T[3];
        for (int i = 0; i < 3; ++i) {
            uint64_t S = acc[4 * (size_t)s + 1 + i];
            uint64_t q = S / M, r = S % M;
            T[i] = (int64_t)(256 * q + (512 * r + M) / (2 * M));
            if (target_q) target_q[3 * (size_t)s + i] = (int32_t)T[i];
        }
        clamp_move(comp, nx, ny, nz, comp[anchor[s]], site_q + 3 * (size_t)s, anchor + s, T);
    }
    free(acc);
    return LOS_OK;
}

/* Lloyd loop with the line-of-sight tessellation: sites start at the centres
 * of the seed voxels (Q8 = 256 x, anchor = seed); T x (VT + update), then a
 * final VT whose dist/src/phi/cell are returned.                            */
int oracle_los_cvt(const uint32_t *comp, int32_t nx, int32_t ny, int32_t nz,
                   const uint32_t *seeds, uint32_t n_sites, const uint16_t *weights, int32_t iters,
                   int32_t *site_q, uint32_t *anchor, double *dist, uint32_t *src, uint32_t *phi,
                   uint32_t *cell) {
    int64_t n;
    int st = los_dims(nx, ny, nz, &n);
    if (st) return st;
    if (iters < 0) return LOS_EINVAL;
    for (uint32_t s = 0; s < n_sites; ++s) {
        if ((int64_t)seeds[s] >= n) return LOS_EINVAL;
        ivec p = coords(seeds[s], nx, ny);
        site_q[3 * (size_t)s + 0] = (int32_t)(256 * p.x);
        site_q[3 * (size_t)s + 1] = (int32_t)(256 * p.y);
        site_q[3 * (size_t)s + 2] = (int32_t)(256 * p.z);
        anchor[s] = seeds[s];
    }
    for (int32_t t = 0; t <= iters; ++t) {
        st = oracle_los_vt(comp, nx, ny, nz, site_q, anchor, n_sites, dist, src, phi, cell, NULL);
        if (st || t == iters) break;
        st = oracle_los_update(comp, nx, ny, nz, weights, cell, phi, n_sites, site_q, anchor, NULL);
        if (st) break;
    }
    return st;
}
