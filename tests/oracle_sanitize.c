/* Driver that runs every entry point of the CPU oracle on small seeded
 * volumes, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitize.py compiles it with the oracle's sources and
 * checks that it exits cleanly).  Test infrastructure only. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_bands(const float *f, int64_t n, const float *iso, int32_t n_iso, uint8_t *band);
int oracle_components(const uint8_t *band, int32_t nx, int32_t ny, int32_t nz, int32_t n_bands, uint32_t *comp,
                      uint32_t *n_comp_out, uint8_t *comp_band, uint64_t *comp_size, uint32_t *comp_first,
                      uint32_t *band_offset);
int oracle_vt(const uint32_t *comp, int32_t nx, int32_t ny, int32_t nz, const uint32_t *sites, uint32_t n_sites,
              uint32_t *cell, uint32_t *dist_out);
int oracle_vt_unpruned(const uint32_t *comp, int32_t nx, int32_t ny, int32_t nz, const uint32_t *sites,
                       uint32_t n_sites, uint32_t *cell, uint32_t *dist_out);
int oracle_update(const uint32_t *cell, int32_t nx, int32_t ny, int32_t nz, const uint16_t *weights, uint32_t *sites,
                  uint32_t n_sites, double *ds_out);
int oracle_cvt(const uint32_t *comp, int32_t nx, int32_t ny, int32_t nz, const uint32_t *seeds, uint32_t n_sites,
               const uint16_t *weights, int32_t iters, uint32_t *cell, uint32_t *sites, uint32_t *site_comp,
               double *mean_ds);
int oracle_stats(const uint32_t *unit, int64_t n, uint32_t n_units, const float *vars, int32_t n_vars,
                 const float *edges, int32_t n_bins, uint64_t *cnt, double *mean, double *m2, float *vmin,
                 float *vmax, uint32_t *hist, double *cov);
int oracle_los_cvt(const uint32_t *comp, int32_t nx, int32_t ny, int32_t nz, const uint32_t *seeds, uint32_t n_sites,
                   const uint16_t *weights, int32_t iters, int32_t *site_q, uint32_t *anchor, double *dist,
                   uint32_t *src, uint32_t *phi, uint32_t *cell);
int64_t oracle_supercover(const int32_t *a, const int32_t *b, int32_t *out, int64_t cap);

static uint64_t rng_state = 88172645463325252ull;
static uint32_t rnd(void) {  /* xorshift64 */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (uint32_t)(rng_state >> 32);
}

#define CHECK(call)                                                         \
    do {                                                                    \
        int rc_ = (call);                                                   \
        if (rc_ != 0) {                                                     \
            fprintf(stderr, "%s returned %d\n", #call, rc_);                \
            exit(2);                                                        \
        }                                                                   \
    } while (0)

static void run(int32_t nx, int32_t ny, int32_t nz, int n_iso, int iters, int m, int bins) {
    const int64_t n = (int64_t)nx * ny * nz;
    float *f = malloc(sizeof(float) * n);
    uint16_t *w = malloc(sizeof(uint16_t) * n);
    for (int64_t i = 0; i < n; ++i) {
        /* smooth plus noise, so that components have some extent */
        int64_t x = i % nx, y = (i / nx) % ny, z = i / ((int64_t)nx * ny);
        f[i] = (float)((x * 7 + y * 5 + z * 3) % 23) + (float)(rnd() % 1000) / 250.0f;
        w[i] = (uint16_t)(rnd() % 65535 + 1);
    }
    float iso[16];
    for (int k = 0; k < n_iso; ++k) iso[k] = 4.0f * (float)(k + 1);
    uint8_t *band = malloc(n);
    CHECK(oracle_bands(f, n, iso, n_iso, band));
    uint32_t *comp = malloc(sizeof(uint32_t) * n), n_comp = 0;
    uint8_t *cb = malloc(n);
    uint64_t *cs = malloc(sizeof(uint64_t) * n);
    uint32_t *cf = malloc(sizeof(uint32_t) * n), *bo = malloc(sizeof(uint32_t) * (n_iso + 2));
    CHECK(oracle_components(band, nx, ny, nz, n_iso + 1, comp, &n_comp, cb, cs, cf, bo));
    /* one site in every component plus a few random ones (duplicates allowed) */
    uint32_t S = n_comp + 6;
    uint32_t *seeds = malloc(sizeof(uint32_t) * S);
    for (uint32_t c = 0; c < n_comp; ++c) seeds[c] = cf[c];
    for (uint32_t k = n_comp; k < S; ++k) seeds[k] = rnd() % (uint32_t)n;
    uint32_t *cell = malloc(sizeof(uint32_t) * n), *dist = malloc(sizeof(uint32_t) * n);
    CHECK(oracle_vt(comp, nx, ny, nz, seeds, S, cell, dist));
    CHECK(oracle_vt_unpruned(comp, nx, ny, nz, seeds, S, cell, dist));
    uint32_t *sites = malloc(sizeof(uint32_t) * S), *sc = malloc(sizeof(uint32_t) * S);
    double *ds = malloc(sizeof(double) * S), *mds = malloc(sizeof(double) * (iters + 1));
    for (uint32_t k = 0; k < S; ++k) sites[k] = seeds[k];
    CHECK(oracle_update(cell, nx, ny, nz, w, sites, S, ds));
    CHECK(oracle_update(cell, nx, ny, nz, NULL, sites, S, ds));
    CHECK(oracle_cvt(comp, nx, ny, nz, seeds, S, w, iters, cell, sites, sc, mds));
    float *vars = malloc(sizeof(float) * n * m), *edges = malloc(sizeof(float) * m * (bins + 1));
    for (int64_t i = 0; i < n * m; ++i) vars[i] = (float)(rnd() % 100000) / 1000.0f - 50.0f;
    for (int j = 0; j < m; ++j)
        for (int b = 0; b <= bins; ++b) edges[j * (bins + 1) + b] = -50.0f + 100.0f * (float)b / (float)bins;
    const int64_t P = (int64_t)m * (m + 1) / 2;
    uint64_t *cnt = malloc(sizeof(uint64_t) * S);
    double *mean = malloc(sizeof(double) * S * m), *m2 = malloc(sizeof(double) * S * m);
    float *vmin = malloc(sizeof(float) * S * m), *vmax = malloc(sizeof(float) * S * m);
    uint32_t *hist = malloc(sizeof(uint32_t) * S * m * bins);
    double *cov = malloc(sizeof(double) * S * P);
    CHECK(oracle_stats(cell, n, S, vars, m, edges, bins, cnt, mean, m2, vmin, vmax, hist, cov));
    CHECK(oracle_stats(cell, n, S, vars, m, NULL, 0, cnt, mean, m2, vmin, vmax, NULL, NULL));
    int32_t *sq = malloc(sizeof(int32_t) * 3 * S);
    uint32_t *anchor = malloc(sizeof(uint32_t) * S), *src = malloc(sizeof(uint32_t) * n);
    uint32_t *phi = malloc(sizeof(uint32_t) * n);
    double *ld = malloc(sizeof(double) * n);
    CHECK(oracle_los_cvt(comp, nx, ny, nz, seeds, S, w, iters, sq, anchor, ld, src, phi, cell));
    int32_t a[3] = {0, 0, 0}, b[3] = {nx - 1, ny - 1, nz - 1};
    int32_t *out = malloc(sizeof(int32_t) * 3 * 4096);
    if (oracle_supercover(a, b, out, 4096) < 1) exit(3);
    free(f); free(w); free(band); free(comp); free(cb); free(cs); free(cf); free(bo); free(seeds); free(cell);
    free(dist); free(sites); free(sc); free(ds); free(mds); free(vars); free(edges); free(cnt); free(mean);
    free(m2); free(vmin); free(vmax); free(hist); free(cov); free(sq); free(anchor); free(src); free(phi);
    free(ld); free(out);
}

int main(void) {
    run(9, 7, 5, 3, 3, 3, 8);
    run(1, 1, 17, 2, 2, 2, 4);
    run(16, 1, 1, 4, 1, 1, 2);
    run(13, 11, 6, 5, 4, 4, 16);
    printf("oracle sanitizer run ok\n");
    return 0;
}
