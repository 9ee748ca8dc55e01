/*
 * lsrvt.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot
 * path of the level-set restricted geodesic Voronoi tessellation of Neuroth
 * et al., "Level Set Restricted Voronoi Tessellation for Large scale Spatial
 * Statistical Analysis":
 *
 *   field --(isobands)--> band --(components)--> comp
 *         --(Lloyd loop of restricted geodesic Voronoi passes)--> cell, sites
 *         --(aggregate)--> per-cell / per-component / per-band statistics
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Volumes are C-order [nz][ny][nx]; voxel (x, y, z) has linear index
 *    i = x + nx*(y + ny*z).  Limits: every extent in 1..32767 and
 *    N = nx*ny*nz <= 2^31 - 1 (LSRVT_ELIMIT otherwise).
 *  - d_* arguments are device pointers owned by the caller; h_* are host
 *    pointers.  The library never allocates device memory: scratch space is
 *    the caller's d_work buffer, sized by the matching *_workspace query, and
 *    must be 256-byte aligned.  A buffer that is too small returns
 *    LSRVT_EWORKSPACE before anything is launched.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    on it; calls return once the work is enqueued, except where a call says
 *    it synchronises the stream.
 *  - Arguments are validated on the host before any launch.  Validation that
 *    needs device data (a seed index out of range) is reported by the calls
 *    that synchronise.  Device or launch failures return LSRVT_EDEVICE.
 *  - Labels, sites, counts, minima, maxima and histograms are bit-exact and
 *    independent of scheduling; floating-point statistics use a fixed
 *    reduction order, so repeated calls give bit-identical results.
 *  - Calls on distinct streams with distinct workspaces may run concurrently.
 */
#ifndef LSRVT_H
#define LSRVT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t nx, ny, nz;
} lsrvt_dims;

enum {
  LSRVT_OK = 0,
  LSRVT_EINVAL = 1,     /* bad argument (dims, isovalues, iters, seed index, sizes) */
  LSRVT_ENAN = 2,       /* the field holds a NaN; band labels are unspecified */
  LSRVT_ECAPACITY = 3,  /* an output table is smaller than the number of entries */
  LSRVT_EWORKSPACE = 4, /* d_work is NULL, misaligned or smaller than required */
  LSRVT_ELIMIT = 5,     /* volume beyond the size limits above */
  LSRVT_EDEVICE = 6     /* a HIP runtime or launch error */
};

/* Label of a voxel whose component holds no site (restricted Voronoi pass). */
#define LSRVT_NONE 0xFFFFFFFFu

/* Flags for lsrvt_aggregate. */
#define LSRVT_STATS_HIST 1u /* fill the histograms (needs d_edges, n_bins >= 1) */
#define LSRVT_STATS_COV 2u  /* fill the co-moment (covariance) arrays */

/* Human-readable name of a status code (static string). */
const char *lsrvt_status_string(int32_t status);

/* Library ABI version (major * 10000 + minor * 100 + patch). */
int32_t lsrvt_version(void);

/* ------------------------------------------------------------------------
 * Isoband classification (Sec. 3.1, the isoband definition
 * B_{a,b} = { v : a < f(v) <= b }).
 *
 * band[i] = #{ k : h_iso[k] < d_field[i] }, i.e. the number of isovalues
 * strictly below the value, so a value equal to an isovalue joins the lower
 * band and the two outer half-open bands are included (n_iso + 1 bands).
 *   d_field  float32[N]           input field (+-inf classify normally)
 *   h_iso    float32[n_iso]       strictly increasing, finite; 0 <= n_iso <= 254
 *   d_band   uint8[N]             output band per voxel
 *   d_status uint32[1] or NULL    cleared, then bit 0 is set if any value is NaN
 * Errors: EINVAL (isovalues not strictly increasing / not finite, n_iso out of
 * range, NULL pointers), ELIMIT.  A NaN is reported only through d_status.
 * Needs no workspace.
 */
int32_t lsrvt_isobands(const float *d_field, lsrvt_dims dims, const float *h_iso, int32_t n_iso,
                       uint8_t *d_band, uint32_t *d_status, void *stream);

/* ------------------------------------------------------------------------
 * Connected components of every isoband (Sec. 3.1: an isoband is the union
 * of components no voxel of which is adjacent to a voxel of another), with
 * 6-connectivity: face neighbours with equal band are joined.
 *
 * Components are numbered in the hierarchical order of the paper's
 * structured layout (Sec. 3.2.4, Fig. 5): by band, then by the smallest
 * linear index of their voxels.
 *   d_band         uint8[N]        band per voxel, every value < n_bands
 *   n_bands        1..255
 *   d_comp         uint32[N]       output component id per voxel
 *   cap_comp       capacity of the four tables below
 *   d_comp_band    uint8[cap_comp]   band of each component
 *   d_comp_size    uint64[cap_comp]  voxel count of each component
 *   d_comp_first   uint32[cap_comp]  smallest linear index in each component
 *   d_band_offset  uint32[n_bands+1] components of band b are
 *                                    [band_offset[b], band_offset[b+1])
 *   h_n_comp       output: number of components
 * Synchronises the stream once (to learn the component count).  If the count
 * exceeds cap_comp, d_comp and *h_n_comp are valid, the tables are not
 * written and LSRVT_ECAPACITY is returned.  A band value >= n_bands gives
 * unspecified labels (it is not checked on the device).
 * Workspace: lsrvt_components_workspace(dims, n_bands).
 */
size_t lsrvt_components_workspace(lsrvt_dims dims, int32_t n_bands);
int32_t lsrvt_components(const uint8_t *d_band, lsrvt_dims dims, int32_t n_bands, uint32_t *d_comp,
                         uint32_t cap_comp, uint8_t *d_comp_band, uint64_t *d_comp_size,
                         uint32_t *d_comp_first, uint32_t *d_band_offset, uint32_t *h_n_comp,
                         void *d_work, size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------
 * One restricted geodesic Voronoi pass (Eq. 1).  The graph geodesic is the
 * hop count in the 6-neighbour graph whose edges join voxels of equal band
 * (which, for searches started inside a component, is the graph of that
 * component); a voxel belongs to the site s of its component that minimises
 * (hop distance, s), so ties go to the lower site id.
 *   d_band    uint8[N]           band per voxel
 *   d_sites   uint32[n_sites]    site voxels (linear indices); id = position
 *   d_cell    uint32[N]          output site id per voxel, LSRVT_NONE when the
 *                                voxel's component holds no site
 * Co-located sites: the lowest id owns the voxel, higher ids get empty cells.
 * Synchronises the stream (to detect convergence).  EINVAL if a site index
 * is >= N.  Workspace: lsrvt_cvt_workspace(dims, n_sites, 0).
 */
int32_t lsrvt_vt(const uint8_t *d_band, lsrvt_dims dims, const uint32_t *d_sites, uint32_t n_sites,
                 uint32_t *d_cell, void *d_work, size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------
 * One site update (Sec. 3.1, "Centroids or Centers of Mass"; Sec. 3.2.3).
 * For each site s: M = sum of weights over its cell and S_a = sum w * a(v)
 * for a in {x, y, z}, exactly in uint64.  If M = 0 the site stays; otherwise
 * it moves to the voxel v of its cell minimising sum_a (M a(v) - S_a)^2
 * (the voxel nearest the weighted centre of mass, compared exactly), ties to
 * the lower linear index.
 *   d_cell     uint32[N]        cells from lsrvt_vt
 *   d_weights  uint16[N] or NULL (NULL = weight 1 everywhere)
 *   d_sites    uint32[n_sites]  in: current sites; out: moved sites
 *   d_ds       float64[n_sites] or NULL: Euclidean move of each site (voxels)
 * Does not synchronise.  Workspace: lsrvt_cvt_workspace(dims, n_sites, 0).
 */
int32_t lsrvt_update(const uint32_t *d_cell, lsrvt_dims dims, const uint16_t *d_weights,
                     uint32_t *d_sites, uint32_t n_sites, double *d_ds, void *d_work,
                     size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------
 * lsrvt_update without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops that forbid
 * allocation).  Same arguments, semantics and results as lsrvt_update; its
 * scratch (per-site sums, fallback list, moved flags: 37 bytes per site) is
 * a fixed device array inside the library, one per GPU, held until the
 * process ends.  Allocates nothing and does not synchronise.
 * Limit: n_sites <= LSRVT_UPDATE_NOALLOC_MAX_SITES, else ELIMIT (nothing is
 * launched).  Every call on one GPU shares that GPU's scratch, so calls that
 * overlap on one GPU (different streams, or host threads) race: serialise
 * them.  The scratch keeps the last call's contents; each call clears what
 * it needs itself.
 */
#define LSRVT_UPDATE_NOALLOC_MAX_SITES (1u << 18)
int32_t lsrvt_update_noalloc(const uint32_t *d_cell, lsrvt_dims dims, const uint16_t *d_weights,
                             uint32_t *d_sites, uint32_t n_sites, double *d_ds, void *stream);

/* ------------------------------------------------------------------------
 * The Lloyd loop of Algorithm 1 with a fixed number of updates:
 * sites_0 = seeds; for t < iters: cells_t = VT(sites_t),
 * sites_{t+1} = update(cells_t); the output cells are VT(sites_iters).
 * (iters + 1 Voronoi passes and iters updates; iters = 0 is the Voronoi
 * tessellation of the seeds.)
 *   d_band, d_comp   band and component id per voxel (lsrvt_components)
 *   d_seeds          uint32[n_sites] initial site voxels; id = position
 *   d_weights        uint16[N] or NULL (uniform)
 *   d_cell           uint32[N] output cells of the final pass
 *   d_sites          uint32[n_sites] output final sites (may alias d_seeds)
 *   d_site_comp      uint32[n_sites] output component of each seed
 *   h_mean_ds        float64[iters] or NULL: mean Euclidean site move of
 *                    each update, in voxel units
 * Synchronises the stream.  Errors: EINVAL (iters < 0, a seed >= N).
 * Workspace: lsrvt_cvt_workspace(dims, n_sites, iters).
 */
size_t lsrvt_cvt_workspace(lsrvt_dims dims, uint32_t n_sites, int32_t iters);
int32_t lsrvt_cvt(const uint8_t *d_band, const uint32_t *d_comp, lsrvt_dims dims,
                  const uint32_t *d_seeds, uint32_t n_sites, const uint16_t *d_weights, int32_t iters,
                  uint32_t *d_cell, uint32_t *d_sites, uint32_t *d_site_comp, double *h_mean_ds,
                  void *d_work, size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Statistics of every cell, merged up the hierarchy cell -> component ->
 * band (Sec. 3.3, "Aggregation"; the hierarchy of Sec. 3.2.4 / Fig. 5).
 *
 * For every unit and variable j: the voxel count n, the mean, the centred
 * sum of squares M2 = sum (x - mean)^2 (population variance = M2 / n), the
 * minimum and maximum, a histogram over caller-given edges, and the centred
 * co-moments C_jk = sum (x_j - mean_j)(x_k - mean_k), j <= k, packed
 * row-major over the upper triangle (m(m+1)/2 entries, C_jj = M2_j).
 * Statistics are unweighted.  Histogram bin of x: the number of interior
 * edges e_1..e_{B-1} that are <= x (below e_0 -> bin 0, >= e_B -> bin B-1).
 * Cells accumulate in float32 with compensated (error-free two-sum) sums of
 * values shifted by the value at the cell's site; the cell -> component ->
 * band merges are pairwise (Chan et al.) in float64, in a fixed order (cells
 * by site id within a component, components by id within a band).
 * Units with n = 0: mean = M2 = C = 0, min = +inf, max = -inf, hist = 0.
 * Variables must be finite.
 *
 * Output arrays (all device, caller-allocated; U = number of units):
 *   n [U] uint64; mean, m2 [U][m]; vmin, vmax [U][m] float32;
 *   hist [U][m][B] uint32 (or NULL); cov [U][m(m+1)/2] (or NULL).
 * Cell level uses float32 mean/m2/cov, components and bands float64.
 *
 *   d_cell        uint32[N]        cells (LSRVT_NONE voxels are skipped)
 *   d_sites       uint32[n_sites]  site voxels (the shift reference)
 *   d_site_comp   uint32[n_sites]  component of each site
 *   d_comp_band   uint8[n_comp]    band of each component
 *   d_vars        float32[m][N]    the variables, one volume after another
 *   d_edges       float32[m][B+1]  increasing edges (needed with HIST)
 *   flags         LSRVT_STATS_HIST | LSRVT_STATS_COV
 * Synchronises the stream twice (to size its work lists).  Errors: EINVAL
 * (m < 1 or > 32, B < 1 with HIST, m * B > 8192, NULL output arrays that the
 * flags require).  Workspace: lsrvt_aggregate_workspace(...); it includes a
 * structured layout of the cells (see lsrvt_layout).
 */
typedef struct {
  uint64_t *n;
  float *mean;
  float *m2;
  float *vmin;
  float *vmax;
  uint32_t *hist;
  float *cov;
} lsrvt_cell_stats;

typedef struct {
  uint64_t *n;
  double *mean;
  double *m2;
  float *vmin;
  float *vmax;
  uint32_t *hist;
  double *cov;
} lsrvt_group_stats;

size_t lsrvt_aggregate_workspace(lsrvt_dims dims, uint32_t n_sites, uint32_t n_comp, int32_t n_bands,
                                 int32_t n_vars, int32_t n_bins, uint32_t flags);
int32_t lsrvt_aggregate(const uint32_t *d_cell, lsrvt_dims dims, const uint32_t *d_sites,
                        const uint32_t *d_site_comp, uint32_t n_sites, const uint8_t *d_comp_band,
                        uint32_t n_comp, int32_t n_bands, const float *d_vars, int32_t n_vars,
                        const float *d_edges, int32_t n_bins, uint32_t flags,
                        const lsrvt_cell_stats *cell, const lsrvt_group_stats *comp,
                        const lsrvt_group_stats *band, void *d_work, size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Joint moments up to fourth order of every cell, merged up the hierarchy
 * cell -> component -> band: the covariance, coskewness and cokurtosis sums
 * that the joint plots compare between raw data and fitted distribution
 * models (Sec. 4.4), over the hierarchy of Sec. 3.2.4 / Fig. 5.
 * For every unit with n voxels and variables x_1..x_m (d = x - mean):
 *   M2[i,j] = sum d_i d_j (i <= j), M3[i,j,k] = sum d_i d_j d_k (i <= j <= k),
 *   M4[i,j,k,l] = sum d_i d_j d_k d_l (i <= j <= k <= l),
 * each packed in lexicographic order of its index tuple (m(m+1)/2,
 * m(m+1)(m+2)/6 and m(m+1)(m+2)(m+3)/24 entries).  Coskewness and
 * cokurtosis are these sums over n times the standard deviations involved.
 * All arithmetic is float64: cells sum products of offsets from the value
 * at the cell's site and convert them to centred sums; components merge
 * their cells (by site id) and bands their components (by id) with
 * pairwise update formulas (Pebay 2008) in a fixed order.  Units with n = 0
 * report zeros.  Voxels labelled LSRVT_NONE are skipped.
 *   output arrays (device, caller-allocated, U units): n [U] uint64,
 *   mean [U][m], m2 [U][P2], m3 [U][P3], m4 [U][P4] float64; cells are
 *   indexed by site id.
 *   d_cell, d_sites, d_site_comp, d_comp_band: as for lsrvt_aggregate
 *   d_vars        float32[m][N], 1 <= m <= 18 (at m = 18: 171, 1140 and 5985
 *                 entries of M2, M3 and M4 per unit)
 * Synchronises the stream (layout sizes, merge work lists).  Errors:
 * EINVAL (m outside 1..18, bands outside 1..255, NULL arrays).
 * Workspace: lsrvt_comoments_workspace(dims, n_sites, n_comp, n_bands, m).
 */
typedef struct {
  uint64_t *n;
  double *mean;
  double *m2;
  double *m3;
  double *m4;
} lsrvt_moments;

size_t lsrvt_comoments_workspace(lsrvt_dims dims, uint32_t n_sites, uint32_t n_comp, int32_t n_bands,
                                 int32_t n_vars);
int32_t lsrvt_comoments(const uint32_t *d_cell, lsrvt_dims dims, const uint32_t *d_sites,
                        const uint32_t *d_site_comp, uint32_t n_sites, const uint8_t *d_comp_band,
                        uint32_t n_comp, int32_t n_bands, const float *d_vars, int32_t n_vars,
                        const lsrvt_moments *cell, const lsrvt_moments *comp, const lsrvt_moments *band,
                        void *d_work, size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Many independent jobs through the whole path in one call (one job = one
 * volume: Sec. 3.1 isobands and components, Algorithm 1, Sec. 3.3 statistics,
 * as the four calls above compute them).  Jobs run on up to n_streams
 * library-created HIP streams (default priority) driven by as many host
 * threads, so small jobs overlap on the device and one job's host waits do
 * not stall the others; every job's outputs are bit-identical to running its
 * four calls alone.  The call waits for work already enqueued on `stream`
 * before starting and returns when every job is done (it synchronises).
 * Per job: inputs as for the single calls (seeds refer to voxels of the
 * job's volume, cap_comp bounds the component count and sizes the component
 * tables and component statistics); outputs are written to the job's
 * buffers, n_comp and status are set (status LSRVT_ECAPACITY when the
 * volume has more components than cap_comp, with d_comp and n_comp valid).
 * Returns LSRVT_OK when every job succeeded, else the first failing job's
 * status.  Workspace: lsrvt_batch_workspace(jobs, n_jobs, n_streams), one
 * slice per stream sized for the largest job.
 */
typedef struct {
  /* inputs */
  lsrvt_dims dims;
  const float *d_field;      /* float32[N] */
  const float *h_iso;        /* host, n_iso increasing finite isovalues (n_iso + 1 bands) */
  int32_t n_iso;
  const uint32_t *d_seeds;   /* uint32[n_sites] */
  uint32_t n_sites;
  const uint16_t *d_weights; /* uint16[N] or NULL */
  int32_t iters;
  const float *d_vars;       /* float32[n_vars][N] */
  int32_t n_vars;
  const float *d_edges;      /* float32[n_vars][n_bins + 1] or NULL */
  int32_t n_bins;
  uint32_t flags;            /* LSRVT_STATS_HIST | LSRVT_STATS_COV */
  uint32_t cap_comp;
  /* outputs (device, caller-allocated) */
  uint8_t *d_band;           /* [N] */
  uint32_t *d_status;        /* [1] NaN flag of the isoband pass */
  uint32_t *d_comp;          /* [N] */
  uint8_t *d_comp_band;      /* [cap_comp] */
  uint64_t *d_comp_size;     /* [cap_comp] */
  uint32_t *d_comp_first;    /* [cap_comp] */
  uint32_t *d_band_offset;   /* [n_iso + 2] */
  uint32_t *d_cell;          /* [N] */
  uint32_t *d_sites;         /* [n_sites] */
  uint32_t *d_site_comp;     /* [n_sites] */
  lsrvt_cell_stats cell;     /* n_sites units */
  lsrvt_group_stats comp;    /* cap_comp units (the first n_comp are written) */
  lsrvt_group_stats band;    /* n_iso + 1 units */
  /* filled by the call */
  uint32_t n_comp;
  int32_t status;
} lsrvt_job;

size_t lsrvt_batch_workspace(const lsrvt_job *jobs, int32_t n_jobs, int32_t n_streams);
int32_t lsrvt_batch_run(lsrvt_job *jobs, int32_t n_jobs, int32_t n_streams, void *d_work,
                        size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Structured hierarchical layout (Sec. 3.2.4, "Data Reduction and Structured
 * Data Layout"; Fig. 5): the voxels that lie in a cell, ordered by band, then
 * component, then cell, then linear index, so that every band, component
 * and cell is one contiguous range addressed by offsets.  Cells of a
 * component are ordered by site id; components must be numbered band-major
 * (as lsrvt_components numbers them).  Voxels labelled LSRVT_NONE (or with a
 * label >= n_sites) are left out.  The linear indices in d_perm are the
 * voxel coordinates of the layout.
 *   d_cell        uint32[N]         cells (lsrvt_cvt)
 *   d_site_comp   uint32[n_sites]   component of each site; values >= n_comp
 *                                   are placed after all components
 *   d_comp_band   uint8[n_comp]     band of each component, nondecreasing
 *   d_perm        uint32[N]         output: the first *h_n_placed entries are
 *                                   the placed voxels in layout order
 *   d_site_order  uint32[n_sites]   output: the site of the k-th cell
 *   d_cell_off    uint32[n_sites+1] output: cell k is perm[cell_off[k] ..
 *                                   cell_off[k+1])
 *   d_comp_off    uint32[n_comp+1]  output: component c is perm[comp_off[c]
 *                                   .. comp_off[c+1])
 *   d_band_off    uint32[n_bands+1] output: band b is perm[band_off[b] ..
 *                                   band_off[b+1])
 *   h_n_placed    output (may be NULL): number of placed voxels
 * Deterministic.  Synchronises the stream twice.
 * Workspace: lsrvt_layout_workspace(dims, n_sites, n_comp).
 */
size_t lsrvt_layout_workspace(lsrvt_dims dims, uint32_t n_sites, uint32_t n_comp);
int32_t lsrvt_layout(const uint32_t *d_cell, lsrvt_dims dims, const uint32_t *d_site_comp,
                     uint32_t n_sites, const uint8_t *d_comp_band, uint32_t n_comp, int32_t n_bands,
                     uint32_t *d_perm, uint32_t *d_site_order, uint32_t *d_cell_off,
                     uint32_t *d_comp_off, uint32_t *d_band_off, uint32_t *h_n_placed, void *d_work,
                     size_t work_bytes, void *stream);

/* Raw-data extraction in layout order: d_out[j][k] = d_vars[j][d_perm[k]]
 * for k < n_placed and j < n_vars (float32, variable-major).  d_perm entries
 * >= N give NaN.  Needs no workspace; does not synchronise. */
int32_t lsrvt_extract(const float *d_vars, int32_t n_vars, lsrvt_dims dims, const uint32_t *d_perm,
                      uint32_t n_placed, float *d_out, void *stream);

/* ------------------------------------------------------------------------
 * Stratified initial sites (Sec. 3.2.1, Eq. 3 and Eq. 4).  Voxel mass
 * m(v) = d_mass_lut[w(v)] (the attraction gamma enters through the table,
 * e.g. round(s * w^gamma)); m = w without a table, m = 1 without weights.
 * Component C gets n_c = max(ceil(m(C) * N / (rho * M)), 1) sites (M the
 * total mass: one site per rho voxels of average mass).  The volume is cut
 * into cubes of edge `block`; the (component, block) pairs of C share its
 * sites by floor(n_c * m(b) / m(C)) plus one each for the largest
 * remainders n_c * m(b) mod m(C), ties to the lower block index.  Inside a
 * pair the n_b sites are placed by systematic sampling proportional to mass
 * over the pair's voxels in linear-index order: site j is the voxel whose
 * cumulative-mass interval holds floor((o + j * m(b)) / n_b), with
 * o = (w0 | w1 << 32) mod m(b) and (w0, w1) the first two words of
 * Philox4x32-10 with key (seed low, seed high) and counter (block index,
 * component, 0, 0).  A voxel heavier than m(b) / n_b may be picked twice
 * (co-located sites are allowed by lsrvt_cvt).  A component of zero mass
 * gets one site, its first voxel.  Sites are numbered by (component, block
 * index, j).  All decisions are exact integer arithmetic: deterministic.
 *   d_comp        uint32[N]        component of every voxel (< n_comp)
 *   d_comp_first  uint32[n_comp]   smallest linear index of each component
 *                                  (as lsrvt_components outputs it)
 *   d_weights     uint16[N] or NULL
 *   d_mass_lut    uint32[65536] or NULL (requires d_weights)
 *   rho           voxels per site, >= 1
 *   block         cube edge, 1..16
 *   cap_pairs     capacity for (component, block) pairs (sizes the
 *                 workspace); *h_n_pairs receives the count
 *   d_sites       uint32[cap_sites] output; *h_n_sites receives the count
 * LSRVT_ECAPACITY when the pairs or the sites exceed their capacity (the
 * counts are reported; sites are not written), LSRVT_EINVAL for bad
 * arguments or a component id >= n_comp, LSRVT_ELIMIT when a site count
 * does not fit 32 bits.  Synchronises the stream twice.
 * Workspace: lsrvt_seed_workspace(dims, n_comp, block, cap_pairs).
 */
size_t lsrvt_seed_workspace(lsrvt_dims dims, uint32_t n_comp, int32_t block, uint32_t cap_pairs);
int32_t lsrvt_seed(const uint32_t *d_comp, const uint32_t *d_comp_first, lsrvt_dims dims, uint32_t n_comp,
                   const uint16_t *d_weights, const uint32_t *d_mass_lut, uint32_t rho, int32_t block,
                   uint64_t seed, uint32_t cap_pairs, uint32_t *d_sites, uint32_t cap_sites, uint32_t *h_n_sites,
                   uint32_t *h_n_pairs, void *d_work, size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Euclidean line-of-sight tessellation (Eq. 1 with the paths of
 * Sec. 3.2.2), the geodesically weighted site update (Eq. 2, Sec. 3.2.3) and
 * their Lloyd loop.
 *
 * Sites are continuous points in fixed point with 8 fraction bits (Q8:
 * x_q = 256 x, int32[S][3], x fastest), each with an anchor voxel whose
 * closed unit cube holds it.  A voxel is the closed unit cube centred on its
 * integer coordinates; a segment is clear when every voxel whose closed
 * cube meets it lies in the component.
 *
 * lsrvt_los_vt: every component voxel v gets a path to a site: src[v] =
 * LSRVT_LOS_SITE | s when v sees site s (the segment from v to the anchor of
 * s is clear; the leg length is |x_v - x_s|), else the voxel u where the path
 * continues (the segment v-u is clear, length |x_v - x_u| + dist[u]).  Paths
 * grow by synchronous sweeps: v looks at each face neighbour w of its
 * component holding a path and considers the path through src(w) (with its
 * ray test), the path through w (dist[w] + 1) and its own path re-measured.
 * Stage 1 allows paths through sites only; stage 2 all three; each stage
 * ends with the first sweep that changes nothing.  A voxel takes a new path
 * only when the shortest valid one is shorter by a relative 2^-40, and then
 * the preferred path within 2^-40 of that one (a site, lowest id, else the
 * lowest voxel index); each anchor starts with the site of smallest
 * (length, id) that sits in it.  Lengths are float64: sqrt of exact integer
 * squared lengths, correctly rounded, so results are deterministic.
 *   d_comp     uint32[N]      component per voxel, LSRVT_NONE outside
 *   d_site_q   int32[S][3]    Q8 positions;  d_anchor uint32[S] anchors
 *   d_dist     float64[N]     out: path length, +inf where no path
 *   d_src      uint32[N]      out: source code, LSRVT_NONE where no path
 *   d_phi      uint32[N]      out: the line-of-sight voxel of the path
 *                             (phi(v) of Eq. 2), LSRVT_NONE where no path
 *   d_cell     uint32[N]      out: the site of phi(v), LSRVT_NONE
 *   h_sweeps   int32[2] or NULL: sweeps run by stage 1 and stage 2
 * LSRVT_EINVAL when an anchor is outside the volume or its component or
 * does not hold its site; LSRVT_ELIMIT for S >= 2^31 or a stage that has not
 * converged after 100000 sweeps.  Synchronises the stream after every batch
 * of 8 sweeps.  Workspace: lsrvt_los_workspace(dims, n_sites).
 *
 * lsrvt_los_update: M = sum m_v and S = sum m_v x_phi(v) over each cell
 * (exact uint64; m_v the uint16 weight, 1 without weights); the target is
 * round-half-up(256 S / M) in Q8.  The site then walks the segment from its
 * position towards the target starting in its anchor, and stops at the first
 * point where the segment touches the closed cube of a voxel outside its
 * component or the volume, among the cubes it can move into (none behind
 * the anchor on an axis it moves along, none beside it on an axis it does
 * not move along); the position becomes x + trunc(t (target - x)) per axis
 * and the anchor the voxel the walk stopped in.  A cell of zero mass keeps
 * its site.  d_site_q and d_anchor are updated in place; d_target_q
 * (int32[S][3] or NULL) receives the targets, INT32_MIN for empty cells.
 * LSRVT_EINVAL for a cell id >= S.  Synchronises the stream once.
 *
 * lsrvt_los_cvt: sites start at the centres of the seed voxels (anchor =
 * seed), then iters x (lsrvt_los_vt + lsrvt_los_update) and a final
 * lsrvt_los_vt whose outputs are returned; *h_sweeps (may be NULL) receives
 * the total number of sweeps.  LSRVT_EINVAL for a seed outside the volume or
 * outside every component.
 */
#define LSRVT_LOS_SITE 0x80000000u
size_t lsrvt_los_workspace(lsrvt_dims dims, uint32_t n_sites);
int32_t lsrvt_los_vt(const uint32_t *d_comp, lsrvt_dims dims, const int32_t *d_site_q, const uint32_t *d_anchor,
                     uint32_t n_sites, double *d_dist, uint32_t *d_src, uint32_t *d_phi, uint32_t *d_cell,
                     int32_t *h_sweeps, void *d_work, size_t work_bytes, void *stream);
int32_t lsrvt_los_update(const uint32_t *d_comp, lsrvt_dims dims, const uint16_t *d_weights,
                         const uint32_t *d_cell, const uint32_t *d_phi, uint32_t n_sites, int32_t *d_site_q,
                         uint32_t *d_anchor, int32_t *d_target_q, void *d_work, size_t work_bytes, void *stream);
int32_t lsrvt_los_cvt(const uint32_t *d_comp, lsrvt_dims dims, const uint32_t *d_seeds, uint32_t n_sites,
                      const uint16_t *d_weights, int32_t iters, int32_t *d_site_q, uint32_t *d_anchor,
                      double *d_dist, uint32_t *d_src, uint32_t *d_phi, uint32_t *d_cell, int32_t *h_sweeps,
                      void *d_work, size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Schedule of the Voronoi passes of lsrvt_vt and lsrvt_cvt (Eq. 1): both
 * compute the same regions bit for bit.
 *   LSRVT_VT_AUTO     the library's choice from the volume and site count
 *                     (the brick relaxation when there are at least 1024
 *                     voxels per site, the level search otherwise)
 *   LSRVT_VT_LEVELS   level-synchronous breadth-first search, one launch per
 *                     level, over 16^3 bricks of bit masks
 *   LSRVT_VT_BRICKS   brick relaxation: rounds of launches over marked 16^3
 *                     bricks, each relaxed to its own fixed point in LDS
 * The setting belongs to the calling host thread (calls from other threads
 * are not affected).  Returns the previous setting, or -1 (and changes
 * nothing) for an unknown value.  The autotuner of the Python package picks
 * it per job class by measurement.
 */
#define LSRVT_VT_AUTO 0
#define LSRVT_VT_LEVELS 1
#define LSRVT_VT_BRICKS 2
int32_t lsrvt_set_vt_engine(int32_t engine);

/* ------------------------------------------------------------------------
 * Launch shapes and schedule choices of the calling host thread's later
 * calls (none of them changes what is computed; the autotuner of the Python
 * package picks the two launch shapes per job class by measurement, the
 * other two are for tests and experiments):
 *   LSRVT_TUNE_BR_GRID      workgroups of each brick-relaxation round
 *                           (each walks the round's bricks with that stride):
 *                           256 .. 16384, 0 = the library's choice (2048)
 *   LSRVT_TUNE_STATS_TILE   voxels staged in LDS per thread and round by the
 *                           statistics' cell kernel (its tile is this times
 *                           its workgroup size): 1, 2 or 4, 0 = the largest
 *                           that keeps a workgroup within 40 KiB of LDS
 *   LSRVT_TUNE_KEY_BITS     key width of the brick relaxation: 0 = narrow
 *                           32-bit keys (distance and site id) when the site
 *                           ids fit in 24 bits, wide 64-bit keys otherwise;
 *                           64 = always wide; 1 .. 30 = narrow with an id
 *                           field of at least that many bits (fewer distance
 *                           bits).  A pass whose distances outgrow the
 *                           narrow field is repeated with wide keys, which
 *                           the rest of the call keeps, so every value gives
 *                           the same results.
 *   LSRVT_TUNE_RESET        how an incremental relaxation pass of lsrvt_cvt
 *                           starts: 0 = the reset of moved sites' voxels is
 *                           fused into the first round (which then works on
 *                           every brick) when the moved sites' cells cover
 *                           most bricks, else done by its own kernel (which
 *                           reads every key but lets the first round work
 *                           only on bricks with reset voxels); 1 = always
 *                           its own kernel; 2 = always fused.
 * Returns the previous value, or -1 (and changes nothing) for an unknown
 * knob or a value outside its range.
 */
#define LSRVT_TUNE_BR_GRID 1
#define LSRVT_TUNE_STATS_TILE 2
#define LSRVT_TUNE_KEY_BITS 3
#define LSRVT_TUNE_RESET 4
int32_t lsrvt_set_tuning(int32_t knob, int32_t value);

/* ------------------------------------------------------------------------
 * Benchmark instrumentation of the Voronoi passes' dominant kernel: the
 * level kernel (one launch per breadth-first level) under LSRVT_VT_LEVELS,
 * the relaxation round (one brick-list launch and one round launch per
 * round) under LSRVT_VT_BRICKS.  While enabled, every batch of back-to-back
 * levels or rounds is bracketed by one hipEvent pair recorded on the stream
 * it is launched on.  lsrvt_timing_read waits for the recorded events and
 * returns, since the previous read: the summed milliseconds of those
 * batches, the number of levels or rounds in them, the number of Voronoi
 * passes they belong to, the voxels of one pass and which schedules ran
 * (bit 0 levels, bit 1 bricks); then it resets the totals.  Any output
 * pointer may be NULL.  The state is per host thread: enabling, recording
 * and reading all refer to the calling thread's own record, so calls made
 * from other threads (other streams) are neither timed nor disturbed.
 */
int32_t lsrvt_timing_enable(int32_t enable);
int32_t lsrvt_timing_read(double *ms, uint64_t *launches, uint64_t *passes, int64_t *voxels_per_pass,
                          int32_t *engines);

#ifdef __cplusplus
}
#endif
#endif /* LSRVT_H */
