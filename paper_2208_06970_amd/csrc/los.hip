// Euclidean line-of-sight Voronoi tessellation and the geodesically weighted
// site update (Sec. 3.1 with Eq. 1 and Eq. 2; Sec. 3.2.2 and Sec. 3.2.3).
//
// State per voxel v: the path length d[v] (float64), its source src[v] (a
// voxel index, or LSRVT_LOS_SITE | s when v sees its site s directly) and,
// after the relaxation, phi[v] (the line-of-sight voxel of the path) and
// cell[v] (the site of phi[v]).  Sites are continuous points kept in fixed
// point with 8 fraction bits plus an anchor voxel.
//
// The relaxation is synchronous: a sweep reads the state the previous sweep
// left and writes proposals; an apply pass then installs the proposals.  A
// sweep re-evaluates a voxel only if something it reads changed in the
// previous sweep (itself, a face neighbour, its source, or the source of a
// face neighbour): every other voxel would recompute exactly what it computed
// before, so the sweep equals a full synchronous sweep.
//
// Rounding makes a path through a voxel on the straight line to the site as
// long as the straight line, or an ulp shorter, so a voxel takes a new path
// only when the shortest valid candidate is shorter by a relative 2^-40, and
// then takes the preferred candidate within 2^-40 of that shortest one (the
// site itself first, by id, else the lowest voxel index).
#include <algorithm>
#include <vector>

#include "common.h"

namespace lsrvt {
namespace {

constexpr uint32_t kSite = LSRVT_LOS_SITE;
constexpr int kLosThreads = 256;
constexpr int kSweepBatch = 8;
constexpr int32_t kMaxSweeps = 100000;
constexpr int kPhiRounds = 40;
constexpr double kShorter = 1.0 - 0x1p-40;
constexpr double kNear = 1.0 + 0x1p-40;
constexpr int kMarkPer = 16;  // voxels per thread in mark and apply (a chunk: 4096 voxels)

struct LosArgs {
  const uint32_t *comp;
  Geom g;
  const int32_t *site_q;  // [S][3] Q8
  const uint32_t *anchor; // [S]
  uint32_t n_sites;
  double *d;              // [N] path lengths (the caller's output)
  uint32_t *src;          // [N] sources (the caller's output)
  double *pd;             // [N] proposed lengths
  uint32_t *ps;           // [N] proposed sources
  uint8_t *chg;           // [N] changed in this sweep
  uint8_t *flag;          // [N] v or its source changed in the sweep before
  uint8_t *chunk_any;     // [chunks] some flag of the chunk is set
  uint32_t *list;         // [N] voxels to evaluate in this sweep
  uint32_t *count;        // length of list
  uint32_t *alive;        // [kSweepBatch] a voxel changed in sweep j of the batch
  uint32_t *err;
};

// Coordinates of voxel v (v < 2^31, so 32-bit division is exact).
__device__ __forceinline__ void xyz(int64_t v, const Geom &g, int32_t &x, int32_t &y, int32_t &z) {
  const uint32_t u = (uint32_t)v, nx = (uint32_t)g.nx, ny = (uint32_t)g.ny;
  const uint32_t row = u / nx;
  const uint32_t zz = row / ny;
  x = (int32_t)(u - row * nx);
  y = (int32_t)(row - zz * ny);
  z = (int32_t)zz;
}

__device__ __forceinline__ double len_vox(int32_t ax, int32_t ay, int32_t az, int32_t bx, int32_t by, int32_t bz) {
  int64_t dx = ax - bx, dy = ay - by, dz = az - bz;
  return sqrt((double)(dx * dx + dy * dy + dz * dz));
}

__device__ __forceinline__ double len_site(int32_t x, int32_t y, int32_t z, const int32_t *q) {
  int64_t dx = 256 * (int64_t)x - q[0], dy = 256 * (int64_t)y - q[1], dz = 256 * (int64_t)z - q[2];
  return sqrt((double)(dx * dx + dy * dy + dz * dz)) / 256.0;
}

// True when every voxel whose closed cube meets the segment between the
// centres of a and b belongs to component c.  Plane crossings of axis i
// happen at t = (2k + 1) / (2 L_i); they are ordered by cross-multiplication
// ((2k + 1) L_j < 2^31 under the extent limit), and at a crossing shared by
// several axes every combination of their steps is touched.  The walk stays
// in the bounding box of a and b, so every read is in bounds.
__device__ bool ray_clear(const uint32_t *__restrict__ comp, const Geom &g, int32_t ax, int32_t ay, int32_t az,
                          int32_t bx, int32_t by, int32_t bz, uint32_t c) {
  const uint32_t L[3] = {(uint32_t)abs(bx - ax), (uint32_t)abs(by - ay), (uint32_t)abs(bz - az)};
  const int64_t stp[3] = {bx > ax ? 1 : -1, (by > ay ? 1 : -1) * (int64_t)g.nx,
                          (bz > az ? 1 : -1) * (int64_t)g.nx * g.ny};
  uint32_t m[3] = {0, 0, 0};
  int64_t cur = ax + (int64_t)g.nx * (ay + (int64_t)g.ny * az);
  for (;;) {
    int best = -1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (m[i] >= L[i]) continue;
      if (best < 0 || (2 * m[i] + 1) * L[best] < (2 * m[best] + 1) * L[i]) best = i;
    }
    if (best < 0) return true;
    uint32_t tied = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (m[i] < L[i] && (2 * m[i] + 1) * L[best] == (2 * m[best] + 1) * L[i]) tied |= 1u << i;
    for (uint32_t sub = tied; sub; sub = (sub - 1) & tied) {
      int64_t q = cur;
      if (sub & 1u) q += stp[0];
      if (sub & 2u) q += stp[1];
      if (sub & 4u) q += stp[2];
      if (comp[q] != c) return false;
    }
    if (tied & 1u) { cur += stp[0]; m[0] += 1; }
    if (tied & 2u) { cur += stp[1]; m[1] += 1; }
    if (tied & 4u) { cur += stp[2]; m[2] += 1; }
  }
}

__device__ __forceinline__ uint32_t pref(uint32_t code) { return code ^ kSite; }

// ---------------------------------------------------------------- anchors
__global__ void k_los_check(const uint32_t *__restrict__ comp, Geom g, const int32_t *__restrict__ q,
                            const uint32_t *__restrict__ anchor, uint32_t S, uint32_t *err) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  uint32_t a = anchor[s];
  if ((int64_t)a >= g.n || comp[a] == kNone) { err[0] = 1u; return; }
  int32_t x, y, z;
  xyz(a, g, x, y, z);
  const int32_t *p = q + 3 * (size_t)s;
  if (abs(256 * x - p[0]) > 128 || abs(256 * y - p[1]) > 128 || abs(256 * z - p[2]) > 128) err[0] = 1u;
}

// Each anchor holds the site with the smallest (length, id): the smallest
// length by an atomic min on its bit pattern (non-negative doubles order as
// their bits), then the smallest id among the sites that reach it.
__global__ void k_anchor_reset(LosArgs A) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= A.n_sites) return;
  uint32_t a = A.anchor[s];
  reinterpret_cast<unsigned long long *>(A.pd)[a] = 0x7FF0000000000000ull;
  A.ps[a] = kNone;
}

__global__ void k_anchor_len(LosArgs A) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= A.n_sites) return;
  uint32_t a = A.anchor[s];
  int32_t x, y, z;
  xyz(a, A.g, x, y, z);
  double d = len_site(x, y, z, A.site_q + 3 * (size_t)s);
  atomicMin(reinterpret_cast<unsigned long long *>(A.pd) + a, (unsigned long long)__double_as_longlong(d));
}

__global__ void k_anchor_id(LosArgs A) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= A.n_sites) return;
  uint32_t a = A.anchor[s];
  int32_t x, y, z;
  xyz(a, A.g, x, y, z);
  double d = len_site(x, y, z, A.site_q + 3 * (size_t)s);
  if (d == A.pd[a]) atomicMin(A.ps + a, s);
}

__global__ void k_anchor_set(LosArgs A) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= A.n_sites) return;
  uint32_t a = A.anchor[s];
  if (A.ps[a] != s) return;
  A.d[a] = A.pd[a];
  A.src[a] = kSite | s;
  A.flag[a] = 1;  // the anchors' neighbourhoods are evaluated in the first sweep
  A.chunk_any[a / ((uint32_t)kLosThreads * kMarkPer)] = 1;
}

// ---------------------------------------------------------------- sweeps
// A sweep is three launches.  mark: every component voxel whose flag or a
// face neighbour's flag is set (or every one, in the first sweep of a stage)
// is listed, and the change plane is cleared.  eval: each listed voxel
// evaluates its candidates against the state of the previous sweep and
// writes a proposal if it changes.  apply: proposals are installed and flag
// is set for each voxel that changed or whose source changed.  A voxel left
// out reads nothing that changed since it was last evaluated, so it would
// compute the same result: the sweep equals a full synchronous sweep.

__global__ void __launch_bounds__(kLosThreads) k_los_mark(LosArgs A, int all_dirty) {
  __shared__ uint32_t part[kLosThreads];
  __shared__ uint32_t base;
  __shared__ uint32_t live;
  const Geom g = A.g;
  const int64_t C = (int64_t)kLosThreads * kMarkPer;
  const int64_t chunk = (int64_t)blockIdx.x * C;
  if (!all_dirty) {
    // A voxel of this chunk can be dirty only if a flag is set in the chunk
    // or in a chunk that holds one of its face neighbours (offsets 1, nx and
    // nx*ny).  Any change of the chunk itself in the sweep before set a flag
    // here, so a skipped chunk has nothing to clear either.
    if (threadIdx.x == 0) {
      const int64_t nch = (g.n + C - 1) / C;
      const int64_t off[3] = {1, g.nx, (int64_t)g.nx * g.ny};
      uint32_t any = A.chunk_any[blockIdx.x];
      for (int k = 0; k < 3 && !any; ++k)
        for (int sgn = -1; sgn <= 1 && !any; sgn += 2) {
          int64_t lo = (chunk + sgn * off[k]) / C, hi = (chunk + C - 1 + sgn * off[k]) / C;
          if (chunk + sgn * off[k] < 0) lo = 0;
          lo = lo < 0 ? 0 : lo;
          hi = hi >= nch ? nch - 1 : hi;
          for (int64_t b = lo; b <= hi && !any; ++b) any = A.chunk_any[b];
        }
      live = any;
    }
    __syncthreads();
    if (!live) return;
  }
  uint32_t bits = 0, cnt = 0;
#pragma unroll 4
  for (int j = 0; j < kMarkPer; ++j) {
    const int64_t v = chunk + (int64_t)j * kLosThreads + threadIdx.x;
    if (v >= g.n) break;
    A.chg[v] = 0;
    if (A.comp[v] == kNone) continue;
    int32_t x, y, z;
    xyz(v, g, x, y, z);
    const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny;
    // every load is issued (clamped to v at the volume's faces), then combined
    const uint32_t f = (uint32_t)A.flag[v] | A.flag[x > 0 ? v - 1 : v] | A.flag[x < g.nx - 1 ? v + 1 : v] |
                       A.flag[y > 0 ? v - sy : v] | A.flag[y < g.ny - 1 ? v + sy : v] |
                       A.flag[z > 0 ? v - sz : v] | A.flag[z < g.nz - 1 ? v + sz : v];
    const bool dirty = all_dirty || f != 0;
    if (dirty) { bits |= 1u << j; ++cnt; }
  }
  // block-wide exclusive scan of the per-thread counts, one atomic per block
  part[threadIdx.x] = cnt;
  __syncthreads();
  for (int o = 1; o < kLosThreads; o <<= 1) {
    const uint32_t t = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0u;
    __syncthreads();
    part[threadIdx.x] += t;
    __syncthreads();
  }
  if (threadIdx.x == kLosThreads - 1) base = part[kLosThreads - 1] ? atomicAdd(A.count, part[kLosThreads - 1]) : 0u;
  __syncthreads();
  uint32_t at = base + part[threadIdx.x] - cnt;
  for (int j = 0; j < kMarkPer && bits; ++j)
    if (bits & (1u << j)) {
      A.list[at++] = (uint32_t)(chunk + (int64_t)j * kLosThreads + threadIdx.x);
      bits &= ~(1u << j);
    }
}

// The segment from voxel (x, y, z) to the ray target of candidate code cc
// (the voxel itself, or the anchor of a site) is clear.
__device__ __forceinline__ bool clear_to(const LosArgs &A, int32_t x, int32_t y, int32_t z, uint32_t cc, uint32_t c) {
  const uint32_t t = (cc & kSite) ? A.anchor[cc & ~kSite] : cc;
  int32_t ux, uy, uz;
  xyz(t, A.g, ux, uy, uz);
  return ray_clear(A.comp, A.g, x, y, z, ux, uy, uz, c);
}

template <int Stage>
__device__ __forceinline__ bool los_eval(const LosArgs &A, uint32_t v) {
  const Geom g = A.g;
  const uint32_t c = A.comp[v];
  int32_t x, y, z;
  xyz(v, g, x, y, z);
  const uint32_t sy = (uint32_t)g.nx, sz = (uint32_t)g.nx * (uint32_t)g.ny;
  const uint32_t sv = A.src[v];
  const double dh = A.d[v];
  // candidates: length cd, source code cc; bit i of need: a ray must be
  // clear; known/ok: validity decided / valid (not shorter counts invalid)
  // Fixed slots, so every index is a compile-time constant: stage 1 has the
  // path through the site of neighbour i in slot i; stage 2 has the path
  // through src(w_i) in slot 2i, through w_i in slot 2i + 1, and the voxel's
  // own path re-measured in slot 12.  Bit i of `have` marks a candidate.
  constexpr int kCand = Stage == 1 ? 6 : 13;
  double cd[kCand];
  uint32_t cc[kCand];
  uint32_t need = 0, have = 0;
#pragma unroll
  for (int i = 0; i < kCand; ++i) { cd[i] = 0.0; cc[i] = 0u; }
  if (Stage == 2 && sv != kNone && !(sv & kSite)) {
    int32_t ux, uy, uz;
    xyz(sv, g, ux, uy, uz);
    cd[kCand - 1] = len_vox(x, y, z, ux, uy, uz) + A.d[sv];
    cc[kCand - 1] = sv;
    have |= 1u << (kCand - 1);
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const bool in = i == 0 ? x > 0 : i == 1 ? x < g.nx - 1 : i == 2 ? y > 0 : i == 3 ? y < g.ny - 1
                  : i == 4 ? z > 0 : z < g.nz - 1;
    if (!in) continue;
    const uint32_t w = i == 0 ? v - 1 : i == 1 ? v + 1 : i == 2 ? v - sy : i == 3 ? v + sy : i == 4 ? v - sz : v + sz;
    if (A.comp[w] != c) continue;
    const uint32_t u = A.src[w];
    if (u == kNone) continue;
    constexpr int kStep = Stage == 1 ? 1 : 2;
    if (u & kSite) {
      cd[kStep * i] = len_site(x, y, z, A.site_q + 3 * (size_t)(u & ~kSite));
      cc[kStep * i] = u;
      need |= 1u << (kStep * i);
      have |= 1u << (kStep * i);
    } else if (Stage == 2 && u != v) {
      int32_t ux, uy, uz;
      xyz(u, g, ux, uy, uz);
      cd[kStep * i] = len_vox(x, y, z, ux, uy, uz) + A.d[u];
      cc[kStep * i] = u;
      need |= 1u << (kStep * i);
      have |= 1u << (kStep * i);
    }
    if (Stage == 2) {
      cd[2 * i + 1] = A.d[w] + 1.0;
      cc[2 * i + 1] = w;
      have |= 1u << (2 * i + 1);
    }
  }
  // Every loop below runs over the compile-time bound kCand (fully
  // unrolled), so the candidate arrays stay in registers.
  uint32_t known = 0, ok = 0;
#pragma unroll
  for (int i = 0; i < kCand; ++i)
    if ((have & (1u << i)) && !(cd[i] < dh)) known |= 1u << i;
  // decides the candidate with code bc and every other undecided one with
  // the same code that needs a ray (the same segment)
  auto decide = [&](int bi, uint32_t bc, bool bneed) {
    bool good = true;
    if (bneed) {
      good = clear_to(A, x, y, z, bc, c);
#pragma unroll
      for (int j = 0; j < kCand; ++j)
        if ((have & (1u << j)) && !(known & (1u << j)) && (need & (1u << j)) && cc[j] == bc) {
          known |= 1u << j;
          if (good) ok |= 1u << j;
        }
    }
    known |= 1u << bi;
    if (good) ok |= 1u << bi;
    return good;
  };
  // the shortest valid candidate, deciding shortest first
  double dmin = __builtin_inf();
  for (;;) {
    int bi = -1;
    double bd = 0.0;
    uint32_t bc = 0;
#pragma unroll
    for (int i = 0; i < kCand; ++i)
      if ((have & (1u << i)) && !(known & (1u << i)) && (bi < 0 || cd[i] < bd)) { bi = i; bd = cd[i]; bc = cc[i]; }
    if (bi < 0) break;
    if (decide(bi, bc, (need >> bi) & 1u)) { dmin = bd; break; }
  }
  if (!(dmin < dh * kShorter)) return false;
  const double lim = dmin * kNear;
  bool got = false;
  double sd = 0.0;
  uint32_t sc = 0;
#pragma unroll
  for (int i = 0; i < kCand; ++i) {
    if (!(have & (1u << i)) || cd[i] > lim) continue;
    if (!(known & (1u << i))) decide(i, cc[i], (need >> i) & 1u);
    if (!(ok & (1u << i))) continue;
    if (!got || pref(cc[i]) < pref(sc) || (cc[i] == sc && cd[i] < sd)) { got = true; sd = cd[i]; sc = cc[i]; }
  }
  A.pd[v] = sd;
  A.ps[v] = sc;
  A.chg[v] = 1;
  return true;
}

// One synchronous sweep of stage 1 (paths only through sites) or stage 2
// over the listed voxels; slot names the sweep in the batch.
template <int Stage>
__global__ void __launch_bounds__(kLosThreads) k_los_eval(LosArgs A, int slot) {
  const uint32_t n = *A.count;
  bool changed = false;
  for (uint32_t i = blockIdx.x * kLosThreads + threadIdx.x; i < n; i += gridDim.x * kLosThreads)
    changed = los_eval<Stage>(A, A.list[i]) || changed;
  if (__ballot(changed) != 0ull && lane_id() == 0) A.alive[slot] = 1u;
}

__global__ void __launch_bounds__(kLosThreads) k_los_apply(LosArgs A) {
  const Geom g = A.g;
  const int64_t chunk = (int64_t)blockIdx.x * kLosThreads * kMarkPer;
  if (blockIdx.x == 0 && threadIdx.x == 0) *A.count = 0u;  // eval of this sweep has finished
  int any = 0;
#pragma unroll 4
  for (int j = 0; j < kMarkPer; ++j) {
    const int64_t v = chunk + (int64_t)j * kLosThreads + threadIdx.x;
    if (v >= g.n) break;
    uint32_t s = A.src[v];
    const uint8_t ch = A.chg[v];
    if (ch) {
      A.d[v] = A.pd[v];
      s = A.ps[v];
      A.src[v] = s;
    }
    const int f = (ch || (s != kNone && !(s & kSite) && A.chg[s])) ? 1 : 0;
    A.flag[v] = (uint8_t)f;
    any |= f;
  }
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) A.chunk_any[blockIdx.x] = any ? 1 : 0;
}

// ---------------------------------------------------------------- phi, cells
__global__ void k_phi_init(const uint32_t *__restrict__ src, int64_t n, uint32_t *__restrict__ phi) {
  const int64_t v = (int64_t)blockIdx.x * kLosThreads + threadIdx.x;
  if (v >= n) return;
  const uint32_t s = src[v];
  phi[v] = s == kNone ? kNone : (s & kSite) ? (uint32_t)v : s;
}

// Pointer jumping towards the line-of-sight voxel of each path; any value
// read (old or new) lies on the same path, so in-place updates are safe.
__global__ void k_phi_jump(const uint32_t *__restrict__ src, int64_t n, uint32_t *phi, uint32_t *flag) {
  const int64_t v = (int64_t)blockIdx.x * kLosThreads + threadIdx.x;
  bool moved = false;
  if (v < n) {
    const uint32_t p = phi[v];
    if (p != kNone && !(src[p] & kSite)) {
      phi[v] = phi[p];
      moved = true;
    }
  }
  if (__ballot(moved) != 0ull && lane_id() == 0) flag[0] = 1u;
}

__global__ void k_phi_cell(const uint32_t *__restrict__ src, const uint32_t *__restrict__ phi, int64_t n,
                           uint32_t *__restrict__ cell) {
  const int64_t v = (int64_t)blockIdx.x * kLosThreads + threadIdx.x;
  if (v >= n) return;
  const uint32_t p = phi[v];
  cell[v] = p == kNone ? kNone : (src[p] & ~kSite);
}

// ---------------------------------------------------------------- update
// M and S = sum m x_phi per site.  One workgroup per 64 x 8 x 8 tile, one
// wave per row of 64 voxels along x: a segmented scan sums each run of equal
// cell, the last lane of a run adds it into an LDS table keyed by cell, and
// the table is flushed with one set of global atomics per distinct cell of
// the tile (a run that finds the table full adds straight to global memory).
// The sums are integers, so the order of the additions does not matter.
constexpr int kAccTX = 64, kAccTY = 8, kAccTZ = 8;
constexpr int kAccCap = 512;

__global__ void __launch_bounds__(256) k_los_accum(const uint32_t *__restrict__ cell,
                                                   const uint32_t *__restrict__ phi,
                                                   const uint16_t *__restrict__ w, Geom g, uint32_t S,
                                                   unsigned long long *acc, uint32_t *err) {
  __shared__ uint32_t tkey[kAccCap];
  __shared__ unsigned long long tM[kAccCap], tX[kAccCap], tY[kAccCap], tZ[kAccCap];
  const int t = threadIdx.x, lane = lane_id(), wid = t / kWave;
  const int ntx = (g.nx + kAccTX - 1) / kAccTX, nty = (g.ny + kAccTY - 1) / kAccTY;
  const int ntz = (g.nz + kAccTZ - 1) / kAccTZ;
  const int64_t ntiles = (int64_t)ntx * nty * ntz;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    for (int i = t; i < kAccCap; i += 256) {
      tkey[i] = kNone;
      tM[i] = tX[i] = tY[i] = tZ[i] = 0ull;
    }
    __syncthreads();
    const int tx = (int)(tile % ntx), ty = (int)((tile / ntx) % nty), tz = (int)(tile / ((int64_t)ntx * nty));
    const int x = tx * kAccTX + lane;
    for (int r = wid; r < kAccTY * kAccTZ; r += 256 / kWave) {
      const int y = ty * kAccTY + (r % kAccTY), z = tz * kAccTZ + (r / kAccTY);
      if (y >= g.ny || z >= g.nz) continue;  // uniform across the wave
      const int64_t v = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
      uint32_t s = x < g.nx ? cell[v] : kNone;
      if (s != kNone && s >= S) {
        err[0] = 1u;
        s = kNone;
      }
      uint64_t m = 0, sx = 0, sy = 0, sz = 0;
      if (s != kNone) {
        m = w ? w[v] : 1u;
        int32_t px, py, pz;
        xyz(phi[v], g, px, py, pz);
        sx = m * (uint64_t)px;
        sy = m * (uint64_t)py;
        sz = m * (uint64_t)pz;
      }
      // segmented inclusive scan; a lane stops adding once its range holds
      // the start of its run
      const uint32_t sl_ = __shfl_up(s, 1, kWave), sr = __shfl_down(s, 1, kWave);
      uint32_t head = (lane == 0 || sl_ != s) ? 1u : 0u;
      const bool tail = lane == kWave - 1 || sr != s;
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t ho = __shfl_up(head, d, kWave);
        const uint64_t mo = __shfl_up(m, d, kWave), xo = __shfl_up(sx, d, kWave);
        const uint64_t yo = __shfl_up(sy, d, kWave), zo = __shfl_up(sz, d, kWave);
        if (lane >= d && !head) { m += mo; sx += xo; sy += yo; sz += zo; head = ho; }
      }
      if (tail && s != kNone && m) {
        const int sl = lds_slot<kAccCap>(tkey, s);
        if (sl >= 0) {
          atomicAdd(&tM[sl], (unsigned long long)m);
          atomicAdd(&tX[sl], (unsigned long long)sx);
          atomicAdd(&tY[sl], (unsigned long long)sy);
          atomicAdd(&tZ[sl], (unsigned long long)sz);
        } else {
          unsigned long long *a = acc + 4 * (size_t)s;
          atomicAdd(a + 0, (unsigned long long)m);
          atomicAdd(a + 1, (unsigned long long)sx);
          atomicAdd(a + 2, (unsigned long long)sy);
          atomicAdd(a + 3, (unsigned long long)sz);
        }
      }
    }
    __syncthreads();
    for (int i = t; i < kAccCap; i += 256) {
      const uint32_t c = tkey[i];
      if (c != kNone && tM[i]) {
        unsigned long long *a = acc + 4 * (size_t)c;
        atomicAdd(a + 0, tM[i]);
        atomicAdd(a + 1, tX[i]);
        atomicAdd(a + 2, tY[i]);
        atomicAdd(a + 3, tZ[i]);
      }
    }
    __syncthreads();
  }
}

// Target X_c = round-half-up(256 S / M) per axis, then the walk from the
// anchor towards it, stopping where the segment first touches the closed
// cube of a voxel outside the component among the cubes it can move into.
__global__ void k_los_move(const uint32_t *__restrict__ comp, Geom g, uint32_t S,
                           const unsigned long long *__restrict__ acc, int32_t *q, uint32_t *anchor,
                           int32_t *target) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const uint64_t M = acc[4 * (size_t)s];
  int32_t *X = q + 3 * (size_t)s;
  if (M == 0) {
    if (target) target[3 * (size_t)s] = target[3 * (size_t)s + 1] = target[3 * (size_t)s + 2] = INT32_MIN;
    return;
  }
  int64_t T[3];
  for (int i = 0; i < 3; ++i) {
    const uint64_t Si = acc[4 * (size_t)s + 1 + i];
    const uint64_t qq = Si / M, r = Si % M;
    T[i] = (int64_t)(256 * qq + (512 * r + M) / (2 * M));
    if (target) target[3 * (size_t)s + i] = (int32_t)T[i];
  }
  const uint32_t a0 = anchor[s];
  const uint32_t c = comp[a0];
  int32_t cv[3];
  xyz(a0, g, cv[0], cv[1], cv[2]);
  const int32_t ext[3] = {g.nx, g.ny, g.nz};
  int64_t D[3], num[3], den[3];
  int32_t step[3];
  bool moving = false;
  for (int i = 0; i < 3; ++i) {
    D[i] = T[i] - X[i];
    step[i] = D[i] > 0 ? 1 : -1;
    den[i] = D[i] < 0 ? -D[i] : D[i];
    num[i] = (256 * (int64_t)cv[i] + 128 * step[i] - X[i]) * step[i];
    moving = moving || D[i] != 0;
  }
  if (!moving) return;
  for (;;) {
    int best = -1;
    for (int i = 0; i < 3; ++i) {
      if (den[i] == 0 || num[i] >= den[i]) continue;
      if (best < 0 || num[i] * den[best] < num[best] * den[i]) best = i;
    }
    if (best < 0) break;
    uint32_t tied = 0;
    for (int i = 0; i < 3; ++i)
      if (den[i] != 0 && num[i] < den[i] && num[i] * den[best] == num[best] * den[i]) tied |= 1u << i;
    bool blocked = false;
    for (uint32_t sub = tied; sub && !blocked; sub = (sub - 1) & tied) {
      int32_t p[3] = {cv[0], cv[1], cv[2]};
      for (int i = 0; i < 3; ++i)
        if (sub & (1u << i)) p[i] += step[i];
      if (p[0] < 0 || p[1] < 0 || p[2] < 0 || p[0] >= ext[0] || p[1] >= ext[1] || p[2] >= ext[2])
        blocked = true;
      else if (comp[p[0] + (int64_t)g.nx * (p[1] + (int64_t)g.ny * p[2])] != c)
        blocked = true;
    }
    if (blocked) {
      const int64_t tn = num[best], td = den[best];
      for (int i = 0; i < 3; ++i) X[i] = (int32_t)(X[i] + (tn * D[i]) / td);
      anchor[s] = (uint32_t)(cv[0] + (int64_t)g.nx * (cv[1] + (int64_t)g.ny * cv[2]));
      return;
    }
    for (int i = 0; i < 3; ++i)
      if (tied & (1u << i)) { cv[i] += step[i]; num[i] += 256; }
  }
  for (int i = 0; i < 3; ++i) X[i] = (int32_t)T[i];
  anchor[s] = (uint32_t)(cv[0] + (int64_t)g.nx * (cv[1] + (int64_t)g.ny * cv[2]));
}

__global__ void k_los_seed(const uint32_t *__restrict__ comp, Geom g, const uint32_t *__restrict__ seeds,
                           uint32_t S, int32_t *q, uint32_t *anchor, uint32_t *err) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const uint32_t v = seeds[s];
  if ((int64_t)v >= g.n || comp[v] == kNone) { err[0] = 1u; return; }
  int32_t x, y, z;
  xyz(v, g, x, y, z);
  q[3 * (size_t)s + 0] = 256 * x;
  q[3 * (size_t)s + 1] = 256 * y;
  q[3 * (size_t)s + 2] = 256 * z;
  anchor[s] = v;
}

// ---------------------------------------------------------------- host side
struct LosWork {
  double *pd;
  uint32_t *ps;
  uint8_t *chg;
  uint8_t *flag;
  uint8_t *chunk_any;
  uint32_t *list;
  uint32_t *ctl;  // [0] err, [1] phi flag, [2..2+kSweepBatch) alive, [2+kSweepBatch] list length
  unsigned long long *acc;
};

template <class C>
void los_layout(C &cv, const Geom &g, uint32_t S, LosWork *W) {
  double *pd = cv.template take<double>((size_t)g.n);
  uint32_t *ps = cv.template take<uint32_t>((size_t)g.n);
  uint8_t *chg = cv.template take<uint8_t>((size_t)g.n);
  uint8_t *flag = cv.template take<uint8_t>((size_t)g.n);
  uint8_t *chunk_any = cv.template take<uint8_t>((size_t)(g.n / ((int64_t)kLosThreads * kMarkPer) + 1));
  uint32_t *list = cv.template take<uint32_t>((size_t)g.n);
  uint32_t *ctl = cv.template take<uint32_t>(64);
  unsigned long long *acc = cv.template take<unsigned long long>(4 * (size_t)(S ? S : 1));
  if (W) *W = LosWork{pd, ps, chg, flag, chunk_any, list, ctl, acc};
}

int32_t read_err(const uint32_t *d_err, hipStream_t s) {
  uint32_t e = 0;
  {
    const int32_t rc_ = read_words(d_err, 1, &e, s);
    if (rc_) return rc_;
  }
  return e ? LSRVT_EINVAL : LSRVT_OK;
}

int32_t los_vt(const uint32_t *d_comp, const Geom &g, const int32_t *d_q, const uint32_t *d_anchor, uint32_t S,
               double *d_dist, uint32_t *d_src, uint32_t *d_phi, uint32_t *d_cell, int32_t *sweeps,
               const LosWork &W, hipStream_t s) {
  int32_t rc;
  const unsigned gs = grid_for(S, 256, 1 << 20);
  const unsigned gv = (unsigned)((g.n + kLosThreads - 1) / kLosThreads);
  LosArgs A{d_comp, g,      d_q,         d_anchor, S, d_dist, d_src, W.pd, W.ps, W.chg, W.flag, W.chunk_any,
            W.list, W.ctl + 2 + kSweepBatch, W.ctl + 2, W.ctl};
  const unsigned gm = (unsigned)((g.n + (int64_t)kLosThreads * kMarkPer - 1) / ((int64_t)kLosThreads * kMarkPer));
  const unsigned ge = 2048;
  if ((rc = fill<uint32_t>(W.ctl, 2, 0u, s))) return rc;
  if (S) {
    hipLaunchKernelGGL(k_los_check, dim3(gs), dim3(256), 0, s, d_comp, g, d_q, d_anchor, S, W.ctl);
    LSRVT_LAUNCHED();
    if ((rc = read_err(W.ctl, s))) return rc;
  }
  if ((rc = fill<double>(d_dist, g.n, __builtin_inf(), s))) return rc;
  if ((rc = fill<uint32_t>(d_src, g.n, kNone, s))) return rc;
  // mark skips chunks with no flag nearby, so it does not clear the change
  // plane everywhere: start every pass with it clear
  if ((rc = fill<uint8_t>(W.chg, g.n, 0, s))) return rc;
  if ((rc = fill<uint8_t>(W.flag, g.n, 0, s))) return rc;
  if ((rc = fill<uint8_t>(W.chunk_any, gm, 0, s))) return rc;
  if ((rc = fill<uint32_t>(W.ctl + 2 + kSweepBatch, 1, 0u, s))) return rc;
  if (S) {
    hipLaunchKernelGGL(k_anchor_reset, dim3(gs), dim3(256), 0, s, A);
    hipLaunchKernelGGL(k_anchor_len, dim3(gs), dim3(256), 0, s, A);
    hipLaunchKernelGGL(k_anchor_id, dim3(gs), dim3(256), 0, s, A);
    hipLaunchKernelGGL(k_anchor_set, dim3(gs), dim3(256), 0, s, A);
    LSRVT_LAUNCHED();
  }
  for (int stage = 1; stage <= 2; ++stage) {
    int32_t done = 0;
    bool first = true;
    for (;;) {
      if (done >= kMaxSweeps) return LSRVT_ELIMIT;
      if ((rc = fill<uint32_t>(W.ctl + 2, kSweepBatch, 0u, s))) return rc;
      for (int j = 0; j < kSweepBatch; ++j) {
        // the first sweep of stage 2 re-evaluates everything: new candidates
        hipLaunchKernelGGL(k_los_mark, dim3(gm), dim3(kLosThreads), 0, s, A, (first && stage == 2) ? 1 : 0);
        if (stage == 1)
          hipLaunchKernelGGL(k_los_eval<1>, dim3(ge), dim3(kLosThreads), 0, s, A, j);
        else
          hipLaunchKernelGGL(k_los_eval<2>, dim3(ge), dim3(kLosThreads), 0, s, A, j);
        hipLaunchKernelGGL(k_los_apply, dim3(gm), dim3(kLosThreads), 0, s, A);
        first = false;
      }
      LSRVT_LAUNCHED();
      uint32_t alive[kSweepBatch];
      {
        const int32_t rc_ = read_words(W.ctl + 2, kSweepBatch, alive, s);
        if (rc_) return rc_;
      }
      int j = 0;
      while (j < kSweepBatch && alive[j]) ++j;
      if (j < kSweepBatch) {  // sweep j changed nothing: the stage has converged
        done += j + 1;
        break;
      }
      done += kSweepBatch;
    }
    if (sweeps) sweeps[stage - 1] = done;
  }
  hipLaunchKernelGGL(k_phi_init, dim3(gv), dim3(kLosThreads), 0, s, d_src, g.n, d_phi);
  LSRVT_LAUNCHED();
  for (int r = 0;; r += 4) {
    if (r >= kPhiRounds) return LSRVT_ELIMIT;
    if ((rc = fill<uint32_t>(W.ctl + 1, 1, 0u, s))) return rc;
    for (int j = 0; j < 4; ++j)
      hipLaunchKernelGGL(k_phi_jump, dim3(gv), dim3(kLosThreads), 0, s, d_src, g.n, d_phi, W.ctl + 1);
    LSRVT_LAUNCHED();
    uint32_t f = 0;
    LSRVT_HIP(hipMemcpyAsync(&f, W.ctl + 1, sizeof(f), hipMemcpyDeviceToHost, s));
    LSRVT_HIP(hipStreamSynchronize(s));
    if (!f) break;
  }
  hipLaunchKernelGGL(k_phi_cell, dim3(gv), dim3(kLosThreads), 0, s, d_src, d_phi, g.n, d_cell);
  LSRVT_LAUNCHED();
  return LSRVT_OK;
}

int32_t los_update(const uint32_t *d_comp, const Geom &g, const uint16_t *d_w, const uint32_t *d_cell,
                   const uint32_t *d_phi, uint32_t S, int32_t *d_q, uint32_t *d_anchor, int32_t *d_target,
                   const LosWork &W, hipStream_t s) {
  int32_t rc;
  if (S == 0) return LSRVT_OK;
  if ((rc = fill<uint32_t>(W.ctl, 1, 0u, s))) return rc;
  if ((rc = fill<unsigned long long>(W.acc, 4 * (int64_t)S, 0ull, s))) return rc;
  const int64_t ntiles = (int64_t)((g.nx + kAccTX - 1) / kAccTX) * ((g.ny + kAccTY - 1) / kAccTY) *
                         ((g.nz + kAccTZ - 1) / kAccTZ);
  hipLaunchKernelGGL(k_los_accum, dim3((unsigned)std::min<int64_t>(ntiles, 65535)), dim3(256), 0, s, d_cell, d_phi,
                     d_w, g, S, W.acc, W.ctl);
  hipLaunchKernelGGL(k_los_move, dim3(grid_for(S, 256, 1 << 20)), dim3(256), 0, s, d_comp, g, S, W.acc, d_q,
                     d_anchor, d_target);
  LSRVT_LAUNCHED();
  return read_err(W.ctl, s);
}

}  // namespace
}  // namespace lsrvt

using namespace lsrvt;

extern "C" size_t lsrvt_los_workspace(lsrvt_dims dims, uint32_t n_sites) {
  Geom g;
  if (make_geom(dims, g) != LSRVT_OK || n_sites >= kSite) return 0;
  Sizer sz;
  los_layout(sz, g, n_sites, nullptr);
  return sz.off;
}

static int32_t los_prepare(lsrvt_dims dims, uint32_t S, void *d_work, size_t work_bytes, Geom &g, LosWork &W) {
  int32_t rc = make_geom(dims, g);
  if (rc) return rc;
  if (S >= kSite) return LSRVT_ELIMIT;
  if ((rc = check_work(d_work, work_bytes, lsrvt_los_workspace(dims, S)))) return rc;
  Carve cv(d_work, work_bytes);
  los_layout(cv, g, S, &W);
  return cv.ok ? LSRVT_OK : LSRVT_EWORKSPACE;
}

extern "C" int32_t lsrvt_los_vt(const uint32_t *d_comp, lsrvt_dims dims, const int32_t *d_site_q,
                                const uint32_t *d_anchor, uint32_t n_sites, double *d_dist, uint32_t *d_src,
                                uint32_t *d_phi, uint32_t *d_cell, int32_t *h_sweeps, void *d_work,
                                size_t work_bytes, void *stream) {
  if (!d_comp || !d_dist || !d_src || !d_phi || !d_cell || (n_sites && (!d_site_q || !d_anchor)))
    return LSRVT_EINVAL;
  Geom g;
  LosWork W;
  int32_t rc = los_prepare(dims, n_sites, d_work, work_bytes, g, W);
  if (rc) return rc;
  return los_vt(d_comp, g, d_site_q, d_anchor, n_sites, d_dist, d_src, d_phi, d_cell, h_sweeps, W,
                as_stream(stream));
}

extern "C" int32_t lsrvt_los_update(const uint32_t *d_comp, lsrvt_dims dims, const uint16_t *d_weights,
                                    const uint32_t *d_cell, const uint32_t *d_phi, uint32_t n_sites,
                                    int32_t *d_site_q, uint32_t *d_anchor, int32_t *d_target_q, void *d_work,
                                    size_t work_bytes, void *stream) {
  if (!d_comp || !d_cell || !d_phi || (n_sites && (!d_site_q || !d_anchor))) return LSRVT_EINVAL;
  Geom g;
  LosWork W;
  int32_t rc = los_prepare(dims, n_sites, d_work, work_bytes, g, W);
  if (rc) return rc;
  return los_update(d_comp, g, d_weights, d_cell, d_phi, n_sites, d_site_q, d_anchor, d_target_q, W,
                    as_stream(stream));
}

extern "C" int32_t lsrvt_los_cvt(const uint32_t *d_comp, lsrvt_dims dims, const uint32_t *d_seeds,
                                 uint32_t n_sites, const uint16_t *d_weights, int32_t iters, int32_t *d_site_q,
                                 uint32_t *d_anchor, double *d_dist, uint32_t *d_src, uint32_t *d_phi,
                                 uint32_t *d_cell, int32_t *h_sweeps, void *d_work, size_t work_bytes,
                                 void *stream) {
  if (!d_comp || !d_dist || !d_src || !d_phi || !d_cell || iters < 0 ||
      (n_sites && (!d_seeds || !d_site_q || !d_anchor)))
    return LSRVT_EINVAL;
  Geom g;
  LosWork W;
  int32_t rc = los_prepare(dims, n_sites, d_work, work_bytes, g, W);
  if (rc) return rc;
  hipStream_t s = as_stream(stream);
  if (h_sweeps) *h_sweeps = 0;
  if (n_sites) {
    if ((rc = fill<uint32_t>(W.ctl, 1, 0u, s))) return rc;
    hipLaunchKernelGGL(k_los_seed, dim3(grid_for(n_sites, 256, 1 << 20)), dim3(256), 0, s, d_comp, g, d_seeds,
                       n_sites, d_site_q, d_anchor, W.ctl);
    LSRVT_LAUNCHED();
    if ((rc = read_err(W.ctl, s))) return rc;
  }
  for (int32_t t = 0; t <= iters; ++t) {
    int32_t sw[2] = {0, 0};
    rc = los_vt(d_comp, g, d_site_q, d_anchor, n_sites, d_dist, d_src, d_phi, d_cell, sw, W, s);
    if (rc) return rc;
    if (h_sweeps) *h_sweeps += sw[0] + sw[1];
    if (t == iters) break;
    rc = los_update(d_comp, g, d_weights, d_cell, d_phi, n_sites, d_site_q, d_anchor, nullptr, W, s);
    if (rc) return rc;
  }
  return LSRVT_OK;
}
