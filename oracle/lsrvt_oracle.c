/*
 * Plain, slow CPU oracle for the level-set restricted geodesic Voronoi
 * tessellation pipeline (Neuroth et al., "Level Set Restricted Voronoi
 * Tessellation for Large scale Spatial Statistical Analysis").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU library
 * is checked against.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it; the GPU library never links, calls
 * or includes anything from here, and this file includes nothing from it.
 *
 * Every function writes out the plain definition it follows, in the order the
 * paper states it, with no blocking, fusion or reordering:
 *   oracle_bands       isoband membership, Sec. 3.1 ("Level Sets, Isobands,
 *                      and Connected Components"): band = #{isovalues < f}
 *   oracle_components  connected components of each isoband, Sec. 3.1, found
 *                      by an explicit-stack depth-first search in raster order
 *   oracle_vt          restricted geodesic Voronoi regions, Eq. 1, with the
 *                      graph geodesic read as the hop count of the 6-neighbour
 *                      graph restricted to the component, ties to the lower
 *                      site id; computed by one pruned BFS per site
 *   oracle_vt_unpruned the same regions by one full BFS per site followed by
 *                      a lexicographic argmin (tiny grids only)
 *   oracle_update      weighted centre of mass of each region (Sec. 3.1,
 *                      "Centroids or Centers of Mass"), in exact integers,
 *                      then moved to the in-region voxel nearest to it
 *   oracle_cvt         Algorithm 1: seeds, then T x (Voronoi pass + update),
 *                      then a final Voronoi pass
 *   oracle_stats       per-unit count, mean, population variance, min, max,
 *                      histogram and covariance (Sec. 3.3 "Aggregation"),
 *                      two-pass in double precision, computed directly from
 *                      the voxels of each unit
 *
 * Limits shared with the library: N = nx*ny*nz <= 2^31-1, every extent
 * <= 32767, weights are uint16.  Under these limits the centroid sums fit in
 * uint64 and the squared snap distances fit in unsigned __int128.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENAN 2
#define OR_ENOMEM 3
#define OR_ELIMIT 4

#define NONE_ID 0xFFFFFFFFu

typedef unsigned __int128 u128;

static int check_dims(int32_t nx, int32_t ny, int32_t nz, int64_t *n_out) {
    if (nx <= 0 || ny <= 0 || nz <= 0) return OR_EINVAL;
    if (nx > 32767 || ny > 32767 || nz > 32767) return OR_ELIMIT;
    int64_t n = (int64_t)nx * ny * nz;
    if (n > 2147483647LL) return OR_ELIMIT;
    *n_out = n;
    return OR_OK;
}

/* Face neighbours of voxel v (linear index x + nx*(y + ny*z)); returns count. */
static int face_neighbours(int64_t v, int32_t nx, int32_t ny, int32_t nz, int64_t out[6]) {
    int64_t x = v % nx;
    int64_t y = (v / nx) % ny;
    int64_t z = v / ((int64_t)nx * ny);
    int k = 0;
    if (x > 0) out[k++] = v - 1;
    if (x < nx - 1) out[k++] = v + 1;
    if (y > 0) out[k++] = v - nx;
    if (y < ny - 1) out[k++] = v + nx;
    if (z > 0) out[k++] = v - (int64_t)nx * ny;
    if (z < nz - 1) out[k++] = v + (int64_t)nx * ny;
    return k;
}

/* ------------------------------------------------------------------------ */
/* Isobands, Sec. 3.1: B_{a,b} = { v : a < f(v) <= b }.  With the isovalues
 * strictly increasing, voxel v lies in band #{ i : iso_i < f(v) }; the two
 * outer, half-open bands are included, giving n_iso + 1 bands.              */
int oracle_bands(const float *f, int64_t n, const float *iso, int32_t n_iso, uint8_t *band) {
    if (n < 0 || n_iso < 0 || n_iso > 254) return OR_EINVAL;
    for (int32_t i = 0; i < n_iso; ++i) {
        if (!isfinite(iso[i])) return OR_EINVAL;
        if (i > 0 && !(iso[i - 1] < iso[i])) return OR_EINVAL;
    }
    int saw_nan = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (isnan(f[v])) {
            saw_nan = 1;
            band[v] = 0;
            continue;
        }
        int b = 0;
        for (int32_t i = 0; i < n_iso; ++i)
            if (iso[i] < f[v]) ++b;
        band[v] = (uint8_t)b;
    }
    return saw_nan ? OR_ENAN : OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Connected components of each isoband, Sec. 3.1: voxels are joined when they
 * are face neighbours with the same band.  Components are discovered by a
 * depth-first search started from every unlabelled voxel in raster order, so
 * provisional ids come out ordered by each component's smallest linear index.
 * They are then renumbered by a stable counting sort on the band, giving the
 * hierarchical order of the structured layout (Sec. 3.2.4, Fig. 5): band
 * first, then smallest member index.
 * Outputs: comp[N]; comp_band/comp_size/comp_first[n_comp] (capacity N);
 * band_offset[n_bands+1].                                                    */
int oracle_components(const uint8_t *band, int32_t nx, int32_t ny, int32_t nz, int32_t n_bands,
                      uint32_t *comp, uint32_t *n_comp_out, uint8_t *comp_band,
                      uint64_t *comp_size, uint32_t *comp_first, uint32_t *band_offset) {
    int64_t n;
    int st = check_dims(nx, ny, nz, &n);
    if (st) return st;
    if (n_bands < 1 || n_bands > 255) return OR_EINVAL;
    for (int64_t v = 0; v < n; ++v)
        if (band[v] >= n_bands) return OR_EINVAL;

    uint32_t *prov = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t *stack = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint8_t *pband = (uint8_t *)malloc(n);
    uint64_t *psize = (uint64_t *)malloc(sizeof(uint64_t) * n);
    uint32_t *pfirst = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t *canon = (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!prov || !stack || !pband || !psize || !pfirst || !canon) {
        free(prov); free(stack); free(pband); free(psize); free(pfirst); free(canon);
        return OR_ENOMEM;
    }
    for (int64_t v = 0; v < n; ++v) prov[v] = NONE_ID;

    uint32_t np = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (prov[v] != NONE_ID) continue;
        uint32_t p = np++;
        pband[p] = band[v];
        pfirst[p] = (uint32_t)v;
        psize[p] = 0;
        int64_t top = 0;
        prov[v] = p;
        stack[top++] = (uint32_t)v;
        while (top > 0) {
            int64_t u = stack[--top];
            psize[p] += 1;
            int64_t nb[6];
            int k = face_neighbours(u, nx, ny, nz, nb);
            for (int i = 0; i < k; ++i) {
                int64_t w = nb[i];
                if (prov[w] == NONE_ID && band[w] == band[u]) {
                    prov[w] = p;
                    stack[top++] = (uint32_t)w;
                }
            }
        }
    }

    /* stable counting sort of the provisional components by band */
    for (int32_t b = 0; b <= n_bands; ++b) band_offset[b] = 0;
    for (uint32_t p = 0; p < np; ++p) band_offset[pband[p] + 1] += 1;
    for (int32_t b = 0; b < n_bands; ++b) band_offset[b + 1] += band_offset[b];
    uint32_t *next = (uint32_t *)malloc(sizeof(uint32_t) * (n_bands + 1));
    for (int32_t b = 0; b < n_bands; ++b) next[b] = band_offset[b];
    for (uint32_t p = 0; p < np; ++p) canon[p] = next[pband[p]]++;
    free(next);

    for (uint32_t p = 0; p < np; ++p) {
        comp_band[canon[p]] = pband[p];
        comp_size[canon[p]] = psize[p];
        comp_first[canon[p]] = pfirst[p];
    }
    for (int64_t v = 0; v < n; ++v) comp[v] = canon[prov[v]];
    *n_comp_out = np;

    free(prov); free(stack); free(pband); free(psize); free(pfirst); free(canon);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Restricted geodesic Voronoi regions, Eq. 1.  For voxel v in component C,
 * its region is the site s of C minimising (gd(v, s), s) lexicographically,
 * where gd is the hop distance in the 6-neighbour graph restricted to C.
 * One breadth-first search per site in increasing id order; a voxel is
 * entered at depth d only if d is strictly smaller than the distance already
 * recorded for it, so an equal distance keeps the lower id.  This pruning
 * never changes the lexicographic minimum: if an earlier site had already
 * reached some voxel p of a shortest path from s to u at no greater depth,
 * that earlier site is at most as far from u as s is, and s cannot win u.
 * A site whose voxel already holds distance 0 (a lower id at the same voxel)
 * starts no search and keeps an empty region.
 * cell[v] = winning site id, or NONE_ID when C holds no site.
 * dist (optional, may be NULL) receives the hop distance (UINT32_MAX if none). */
int oracle_vt(const uint32_t *comp, int32_t nx, int32_t ny, int32_t nz,
              const uint32_t *sites, uint32_t n_sites, uint32_t *cell, uint32_t *dist_out) {
    int64_t n;
    int st = check_dims(nx, ny, nz, &n);
    if (st) return st;
    for (uint32_t s = 0; s < n_sites; ++s)
        if ((int64_t)sites[s] >= n) return OR_EINVAL;

    uint32_t *dist = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t *queue = (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!dist || !queue) { free(dist); free(queue); return OR_ENOMEM; }
    for (int64_t v = 0; v < n; ++v) { dist[v] = UINT32_MAX; cell[v] = NONE_ID; }

    for (uint32_t s = 0; s < n_sites; ++s) {
        int64_t src = sites[s];
        if (dist[src] == 0) continue;           /* co-located with a lower id */
        int64_t head = 0, tail = 0;
        dist[src] = 0;
        cell[src] = s;
        queue[tail++] = (uint32_t)src;
        while (head < tail) {
            int64_t u = queue[head++];
            uint32_t d = dist[u];
            int64_t nb[6];
            int k = face_neighbours(u, nx, ny, nz, nb);
            for (int i = 0; i < k; ++i) {
                int64_t w = nb[i];
                if (comp[w] != comp[u]) continue;
                if (d + 1 < dist[w]) {
                    dist[w] = d + 1;
                    cell[w] = s;
                    queue[tail++] = (uint32_t)w;
                }
            }
        }
    }
    if (dist_out) memcpy(dist_out, dist, sizeof(uint32_t) * n);
    free(dist);
    free(queue);
    return OR_OK;
}

/* The same regions without pruning: a complete BFS from every site, then the
 * lexicographic argmin of (distance, id) per voxel.  O(S * N); tiny grids.   */
int oracle_vt_unpruned(const uint32_t *comp, int32_t nx, int32_t ny, int32_t nz,
                       const uint32_t *sites, uint32_t n_sites, uint32_t *cell, uint32_t *dist_out) {
    int64_t n;
    int st = check_dims(nx, ny, nz, &n);
    if (st) return st;
    for (uint32_t s = 0; s < n_sites; ++s)
        if ((int64_t)sites[s] >= n) return OR_EINVAL;
    uint32_t *d = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t *best = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t *queue = (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!d || !best || !queue) { free(d); free(best); free(queue); return OR_ENOMEM; }
    for (int64_t v = 0; v < n; ++v) { best[v] = UINT32_MAX; cell[v] = NONE_ID; }
    for (uint32_t s = 0; s < n_sites; ++s) {
        for (int64_t v = 0; v < n; ++v) d[v] = UINT32_MAX;
        int64_t head = 0, tail = 0;
        d[sites[s]] = 0;
        queue[tail++] = sites[s];
        while (head < tail) {
            int64_t u = queue[head++];
            int64_t nb[6];
            int k = face_neighbours(u, nx, ny, nz, nb);
            for (int i = 0; i < k; ++i) {
                int64_t w = nb[i];
                if (comp[w] == comp[u] && d[w] == UINT32_MAX) {
                    d[w] = d[u] + 1;
                    queue[tail++] = (uint32_t)w;
                }
            }
        }
        for (int64_t v = 0; v < n; ++v) {
            /* lexicographic (distance, id): ids arrive in increasing order,
               so only a strictly smaller distance replaces the holder */
            if (d[v] < best[v]) { best[v] = d[v]; cell[v] = s; }
        }
    }
    if (dist_out) memcpy(dist_out, best, sizeof(uint32_t) * n);
    free(d); free(best); free(queue);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Site update, Sec. 3.1 "Centroids or Centers of Mass": the weighted centre of
 * mass of region R_s is (1/M) sum_{v in R_s} m_v x_v with M = sum m_v.  Kept
 * exact: M and the three coordinate moments S_a = sum m_v a(v) are uint64.
 * The site then moves to the voxel of R_s nearest to the centre of mass,
 * i.e. the argmin over v in R_s of  D(v) = sum_a (M a(v) - S_a)^2  (which is
 * M^2 times the squared Euclidean distance), with ties to the lower linear
 * index; D is evaluated in unsigned 128-bit arithmetic.  A region with M = 0
 * (empty, or zero total weight) keeps its site.
 * weights == NULL means m_v = 1.  ds_out[s] receives the Euclidean length of
 * the move in voxel units.                                                    */
int oracle_update(const uint32_t *cell, int32_t nx, int32_t ny, int32_t nz,
                  const uint16_t *weights, uint32_t *sites, uint32_t n_sites, double *ds_out) {
    int64_t n;
    int st = check_dims(nx, ny, nz, &n);
    if (st) return st;
    uint64_t *M = (uint64_t *)calloc(n_sites ? n_sites : 1, sizeof(uint64_t));
    uint64_t *Sx = (uint64_t *)calloc(n_sites ? n_sites : 1, sizeof(uint64_t));
    uint64_t *Sy = (uint64_t *)calloc(n_sites ? n_sites : 1, sizeof(uint64_t));
    uint64_t *Sz = (uint64_t *)calloc(n_sites ? n_sites : 1, sizeof(uint64_t));
    uint64_t *count = (uint64_t *)calloc((size_t)n_sites + 1, sizeof(uint64_t));
    uint32_t *members = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    uint64_t *fill = (uint64_t *)calloc(n_sites ? n_sites : 1, sizeof(uint64_t));
    if (!M || !Sx || !Sy || !Sz || !count || !members || !fill) {
        free(M); free(Sx); free(Sy); free(Sz); free(count); free(members); free(fill);
        return OR_ENOMEM;
    }
    /* moments of every region */
    for (int64_t v = 0; v < n; ++v) {
        uint32_t c = cell[v];
        if (c == NONE_ID) continue;
        if (c >= n_sites) { st = OR_EINVAL; break; }
        uint64_t w = weights ? weights[v] : 1u;
        uint64_t x = (uint64_t)(v % nx), y = (uint64_t)((v / nx) % ny), z = (uint64_t)(v / ((int64_t)nx * ny));
        M[c] += w;
        Sx[c] += w * x;
        Sy[c] += w * y;
        Sz[c] += w * z;
        count[c + 1] += 1;
    }
    if (st == OR_OK) {
        /* list the voxels of every region (counting sort by region id) */
        for (uint32_t s = 0; s < n_sites; ++s) count[s + 1] += count[s];
        for (int64_t v = 0; v < n; ++v) {
            uint32_t c = cell[v];
            if (c == NONE_ID) continue;
            members[count[c] + fill[c]++] = (uint32_t)v;
        }
        for (uint32_t s = 0; s < n_sites; ++s) {
            uint32_t old = sites[s];
            uint32_t nw = old;
            if (M[s] != 0) {
                u128 bestD = 0;
                int have = 0;
                for (uint64_t i = count[s]; i < count[s + 1]; ++i) {
                    int64_t v = members[i];
                    int64_t a[3] = {v % nx, (v / nx) % ny, v / ((int64_t)nx * ny)};
                    uint64_t S[3] = {Sx[s], Sy[s], Sz[s]};
                    u128 D = 0;
                    for (int k = 0; k < 3; ++k) {
                        u128 ma = (u128)M[s] * (u128)(uint64_t)a[k];
                        u128 diff = ma >= S[k] ? ma - S[k] : S[k] - ma;
                        D += diff * diff;
                    }
                    /* members are listed in increasing linear index, so a strict
                       comparison keeps the lower index on ties */
                    if (!have || D < bestD) { bestD = D; nw = (uint32_t)v; have = 1; }
                }
            }
            if (ds_out) {
                double dx = (double)((int64_t)(nw % nx) - (int64_t)(old % nx));
                double dy = (double)((int64_t)((nw / nx) % ny) - (int64_t)((old / nx) % ny));
                double dz = (double)((int64_t)(nw / ((int64_t)nx * ny)) - (int64_t)(old / ((int64_t)nx * ny)));
                ds_out[s] = sqrt(dx * dx + dy * dy + dz * dz);
            }
            sites[s] = nw;
        }
    }
    free(M); free(Sx); free(Sy); free(Sz); free(count); free(members); free(fill);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 with a fixed number of updates T: sites_0 = seeds; for t < T,
 * cells_t = VT(sites_t) and sites_{t+1} = update(cells_t); the output cells
 * are VT(sites_T).  T + 1 Voronoi passes and T updates; T = 0 is the Voronoi
 * tessellation of the seeds.  mean_ds[t] is the mean over all sites of the
 * Euclidean move of update t (voxel units).  site_comp[s] = comp of seed s.  */
int oracle_cvt(const uint32_t *comp, int32_t nx, int32_t ny, int32_t nz,
               const uint32_t *seeds, uint32_t n_sites, const uint16_t *weights, int32_t iters,
               uint32_t *cell, uint32_t *sites, uint32_t *site_comp, double *mean_ds) {
    int64_t n;
    int st = check_dims(nx, ny, nz, &n);
    if (st) return st;
    if (iters < 0) return OR_EINVAL;
    for (uint32_t s = 0; s < n_sites; ++s)
        if ((int64_t)seeds[s] >= n) return OR_EINVAL;
    for (uint32_t s = 0; s < n_sites; ++s) {
        sites[s] = seeds[s];
        site_comp[s] = comp[seeds[s]];
    }
    double *ds = (double *)malloc(sizeof(double) * (n_sites ? n_sites : 1));
    if (!ds) return OR_ENOMEM;
    for (int32_t t = 0; t <= iters; ++t) {
        st = oracle_vt(comp, nx, ny, nz, sites, n_sites, cell, NULL);
        if (st) break;
        if (t == iters) break;
        st = oracle_update(cell, nx, ny, nz, weights, sites, n_sites, ds);
        if (st) break;
        double sum = 0.0;
        for (uint32_t s = 0; s < n_sites; ++s) sum += ds[s];
        if (mean_ds) mean_ds[t] = n_sites ? sum / (double)n_sites : 0.0;
    }
    free(ds);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Statistics of every unit (a cell, a component or a band), Sec. 3.3
 * "Aggregation": count, mean, M2 = sum (x - mean)^2 (population variance is
 * M2 / n), min, max, a histogram with caller-given edges, and the co-moments
 * C_jk = sum (x_j - mean_j)(x_k - mean_k) for j <= k, packed row-major over
 * the upper triangle.  Two passes in double: means first, then the centred
 * sums.  Histogram bin of x: the number of interior edges e_1..e_{B-1} that
 * are <= x (values below e_0 land in bin 0, values >= e_B in bin B-1).
 * unit[v] == NONE_ID skips voxel v.  vars is [n_vars][N].  Empty units get
 * n = 0, mean = M2 = cov = 0, min = +inf, max = -inf, hist = 0.
 * edges, hist and cov may be NULL.                                           */
int oracle_stats(const uint32_t *unit, int64_t n, uint32_t n_units, const float *vars, int32_t n_vars,
                 const float *edges, int32_t n_bins, uint64_t *cnt, double *mean, double *m2,
                 float *vmin, float *vmax, uint32_t *hist, double *cov) {
    if (n_vars < 0 || n_bins < 0) return OR_EINVAL;
    int64_t P = (int64_t)n_vars * (n_vars + 1) / 2;
    for (uint32_t u = 0; u < n_units; ++u) {
        cnt[u] = 0;
        for (int32_t j = 0; j < n_vars; ++j) {
            mean[(int64_t)u * n_vars + j] = 0.0;
            m2[(int64_t)u * n_vars + j] = 0.0;
            vmin[(int64_t)u * n_vars + j] = INFINITY;
            vmax[(int64_t)u * n_vars + j] = -INFINITY;
            if (hist)
                for (int32_t b = 0; b < n_bins; ++b) hist[((int64_t)u * n_vars + j) * n_bins + b] = 0;
        }
        if (cov)
            for (int64_t p = 0; p < P; ++p) cov[(int64_t)u * P + p] = 0.0;
    }
    for (int64_t v = 0; v < n; ++v) {
        uint32_t u = unit[v];
        if (u == NONE_ID) continue;
        if (u >= n_units) return OR_EINVAL;
    }
    /* pass 1: counts, sums, min, max, histograms */
    for (int64_t v = 0; v < n; ++v) {
        uint32_t u = unit[v];
        if (u == NONE_ID) continue;
        cnt[u] += 1;
        for (int32_t j = 0; j < n_vars; ++j) {
            float x = vars[(int64_t)j * n + v];
            int64_t o = (int64_t)u * n_vars + j;
            mean[o] += (double)x;
            if (x < vmin[o]) vmin[o] = x;
            if (x > vmax[o]) vmax[o] = x;
            if (hist && edges && n_bins > 0) {
                const float *e = edges + (int64_t)j * (n_bins + 1);
                int32_t b = 0;
                for (int32_t i = 1; i < n_bins; ++i)
                    if (e[i] <= x) ++b;
                hist[o * n_bins + b] += 1;
            }
        }
    }
    for (uint32_t u = 0; u < n_units; ++u)
        for (int32_t j = 0; j < n_vars; ++j)
            if (cnt[u]) mean[(int64_t)u * n_vars + j] /= (double)cnt[u];
    /* pass 2: centred second moments */
    for (int64_t v = 0; v < n; ++v) {
        uint32_t u = unit[v];
        if (u == NONE_ID) continue;
        int64_t p = 0;
        for (int32_t j = 0; j < n_vars; ++j) {
            double dj = (double)vars[(int64_t)j * n + v] - mean[(int64_t)u * n_vars + j];
            m2[(int64_t)u * n_vars + j] += dj * dj;
            if (cov) {
                for (int32_t k = j; k < n_vars; ++k) {
                    double dk = (double)vars[(int64_t)k * n + v] - mean[(int64_t)u * n_vars + k];
                    cov[(int64_t)u * P + p] += dj * dk;
                    ++p;
                }
            }
        }
    }
    return OR_OK;
}
