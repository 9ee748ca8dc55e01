// Restricted geodesic Voronoi pass (Eq. 1), snapped centroid update (Sec. 3.1
// "Centroids"; Sec. 3.2.3) and the fixed-iteration Lloyd loop (Algorithm 1).
//
// Voronoi pass.  The regions of Eq. 1 with ties to the lower id are computed
// by a breadth-first search restricted to same-band face edges, run level
// by level over the whole volume.  Level 0 holds the sites; at level L every
// voxel not reached yet that has a same-band neighbour reached at level L - 1
// takes the smallest site id among those neighbours.  By induction a voxel
// at hop distance L from its nearest sites receives exactly the smallest of
// their ids: each such site reaches it through a neighbour at distance L - 1
// whose own id is no larger, and every neighbour's id names a site within
// distance L.  Each level is one launch, so the ids of level L - 1 are final
// when level L reads them and the result does not depend on scheduling.
//
// The volume is cut into 16^3 bricks.  Per brick row (16 voxels along x) the
// search keeps three 16-bit masks in global memory: the same-band edges in
// each direction (built once per call, since bands do not change), the
// voxels reached so far and the frontier of the last two levels.  A level
// launch visits only the bricks listed for it, one workgroup per brick and
// one thread per row; a brick that reached anything lists itself and its six
// neighbours for the next level.  Frontier rows of bricks that were not
// visited at a level are stale, but only hold voxels whose neighbours were
// all reached one level after them, so they are masked off by the reached
// mask.  Each voxel is written once per pass.
//
// Update.  Per site, M = sum w and S_a = sum w a are exact uint64 sums
// (per-tile LDS aggregation, then one global atomic per distinct cell).  The nearest lattice point to S/M with ties
// rounded down, q_a = floor((2 S_a + M - 1) / (2 M)), is the answer whenever
// it lies in the cell (it then minimises the distance over all lattice
// points, and among tied points the all-lower corner has the smallest linear
// index).  Otherwise one workgroup searches cubes of growing half-width r
// around q; voxels outside the cube are at least r + 1/2 from the centroid,
// so the search stops once 4 D_best < (M (2 r + 1))^2, comparing
// D = sum_a (M a - S_a)^2 exactly in 128 bits.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <mutex>
#include <utility>
#include <vector>

#include "common.h"

namespace lsrvt {

namespace {

constexpr int BX = 16, BY = 16, BZ = 16;
constexpr int kRows = BY * BZ;  // a brick is 256 rows of 16 voxels along x
constexpr int kVTThreads = 256;
constexpr int kHistLen = 8192;  // per-level record of active brick counts
constexpr int kSub = 64;        // sub-lists per level, so that list appends rarely share a counter

struct VTGrid {
  int32_t nbx, nby, nbz;
  int64_t nbricks;
};

// Global level-synchronous BFS state.  Brick b, row r (y = r & 15,
// z = r >> 4) holds 16 voxels along x as the low 16 bits of a word.
struct BFSArgs {
  Geom g;
  VTGrid bg;
  const uint32_t *eq;  // [nbricks][256][3]: (x- | x+ << 16), (y- | y+ << 16), (z- | z+ << 16) same-band bits
  uint32_t *fr;        // [2][nbricks][256] voxels reached at the previous / current level
  uint32_t *vis;       // [nbricks][256] voxels reached so far
  uint32_t *cell;      // [N] site id of every reached voxel (NONE elsewhere)
  uint32_t *queued;    // [nbricks] tag of the last level a brick was queued for
  uint32_t *list0, *list1;  // bricks of even / odd levels
  uint32_t *cnt;       // [3][kSub] rotating list counters: cnt[L % 3][j] bricks in sub-list j of level L
  uint32_t *hist;      // [kHistLen] active bricks per level
  uint32_t *err;
};

__device__ __forceinline__ int64_t brick_row_base(const Geom &g, int x0, int y, int z) {
  return x0 + (int64_t)g.nx * (y + (int64_t)g.ny * z);
}

// Queue brick (bx, by, bz) (bit 0 of `which`) and its neighbours at x-, x+,
// y-, y+, z-, z+ (bits 1..6) for the level tagged `tag` into sub-list `j`
// (list + j * nbricks, counter cnt[j]): lanes 0..6 of the calling wave take
// one brick each, so the tag atomics overlap.  Called by a whole wave.
__device__ void queue_around(const BFSArgs &A, int bx, int by, int bz, uint32_t tag, uint32_t *list, uint32_t *cnt,
                             uint32_t j, uint32_t which) {
  const int k = lane_id();
  bool want = false;
  uint32_t nb = 0;
  if (k < 7 && ((which >> k) & 1u)) {
    const int nx = bx + (k == 1 ? -1 : k == 2 ? 1 : 0);
    const int ny = by + (k == 3 ? -1 : k == 4 ? 1 : 0);
    const int nz = bz + (k == 5 ? -1 : k == 6 ? 1 : 0);
    if (nx >= 0 && ny >= 0 && nz >= 0 && nx < A.bg.nbx && ny < A.bg.nby && nz < A.bg.nbz) {
      nb = (uint32_t)(nx + A.bg.nbx * (ny + A.bg.nby * nz));
      want = A.queued[nb] < tag && atomicMax(&A.queued[nb], tag) < tag;
    }
  }
  const uint64_t m = __ballot(want);
  if (!m) return;
  uint32_t base = 0;
  if (k == 0) base = atomicAdd(&cnt[j], (uint32_t)__popcll(m));
  base = __shfl(base, 0, kWave);
  if (want) list[(size_t)j * A.bg.nbricks + base + (uint32_t)__popcll(m & lanemask_lt())] = nb;
}

// Per-thread variant for the sites of level 0.
__device__ void queue_around_one(const BFSArgs &A, int bx, int by, int bz, uint32_t tag, uint32_t *list,
                                 uint32_t *cnt, uint32_t j) {
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const int nx = bx + (k == 1 ? -1 : k == 2 ? 1 : 0);
    const int ny = by + (k == 3 ? -1 : k == 4 ? 1 : 0);
    const int nz = bz + (k == 5 ? -1 : k == 6 ? 1 : 0);
    if (nx < 0 || ny < 0 || nz < 0 || nx >= A.bg.nbx || ny >= A.bg.nby || nz >= A.bg.nbz) continue;
    const uint32_t nb = (uint32_t)(nx + A.bg.nbx * (ny + A.bg.nby * nz));
    if (A.queued[nb] < tag && atomicMax(&A.queued[nb], tag) < tag)
      list[(size_t)j * A.bg.nbricks + atomicAdd(&cnt[j], 1u)] = nb;
  }
}

// Same-band masks of every row toward its six neighbours (across brick faces
// too); voxels outside the volume have no edges.  One voxel per lane, so a
// wave covers four rows of a brick and the band reads are coalesced.  Bands
// do not change during a Lloyd loop, so this runs once per call.
__global__ __launch_bounds__(kVTThreads) void k_vt_eq(const uint8_t *__restrict__ band, Geom g, VTGrid bg,
                                                      uint32_t *__restrict__ eq) {
  const int64_t slots = bg.nbricks * kRows * BX;
  const int lane = lane_id();
  const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i - lane < slots;
       i += (int64_t)gridDim.x * blockDim.x) {
    bool p[6] = {false, false, false, false, false, false};
    const int64_t row = i >> 4;  // brick * 256 + (ly + 16 lz)
    if (i < slots) {
      const int64_t b = row / kRows;
      const int t = (int)(row % kRows);
      const int bx = (int)(b % bg.nbx), by = (int)((b / bg.nbx) % bg.nby), bz = (int)(b / ((int64_t)bg.nbx * bg.nby));
      const int x = bx * BX + (int)(i & 15), y = by * BY + (t & 15), z = bz * BZ + (t >> 4);
      if (x < g.nx && y < g.ny && z < g.nz) {
        const int64_t v = x + sy * y + sz * z;
        const uint8_t bv = band[v];
        p[0] = x > 0 && band[v - 1] == bv;
        p[1] = x + 1 < g.nx && band[v + 1] == bv;
        p[2] = y > 0 && band[v - sy] == bv;
        p[3] = y + 1 < g.ny && band[v + sy] == bv;
        p[4] = z > 0 && band[v - sz] == bv;
        p[5] = z + 1 < g.nz && band[v + sz] == bv;
      }
    }
    uint64_t m[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) m[k] = __ballot(p[k]);
    if (i < slots && (lane & 15) == 0) {
      const int sh = lane;  // this lane's row occupies ballot bits sh .. sh + 15
      uint32_t *dst = eq + row * 3;
      dst[0] = (uint32_t)((m[0] >> sh) & 0xFFFFu) | ((uint32_t)((m[1] >> sh) & 0xFFFFu) << 16);
      dst[1] = (uint32_t)((m[2] >> sh) & 0xFFFFu) | ((uint32_t)((m[3] >> sh) & 0xFFFFu) << 16);
      dst[2] = (uint32_t)((m[4] >> sh) & 0xFFFFu) | ((uint32_t)((m[5] >> sh) & 0xFFFFu) << 16);
    }
  }
}

// Level 0: every site reaches its own voxel; co-located sites keep the lowest id.
__global__ void k_bfs_init(const uint32_t *__restrict__ sites, uint32_t S, BFSArgs A, uint32_t tag) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  uint32_t v = sites[s];
  if ((int64_t)v >= A.g.n) {
    atomicOr(A.err, 1u);
    return;
  }
  uint32_t x = v % (uint32_t)A.g.nx, r = v / (uint32_t)A.g.nx;
  uint32_t y = r % (uint32_t)A.g.ny, z = r / (uint32_t)A.g.ny;
  int bx = x / BX, by = y / BY, bz = z / BZ;
  uint32_t b = bx + A.bg.nbx * (by + A.bg.nby * bz);
  uint32_t row = (y % BY) + BY * (z % BZ), bit = 1u << (x % BX);
  atomicMin(&A.cell[v], s);
  atomicOr(&A.vis[(int64_t)b * kRows + row], bit);
  atomicOr(&A.fr[(int64_t)b * kRows + row], bit);  // parity 0 = level 0
  queue_around_one(A, bx, by, bz, tag, A.list1, A.cnt + kSub, blockIdx.x % kSub);
}

// Level L: a voxel not reached yet is reached now when a same-band face
// neighbour was reached at level L - 1; it takes the smallest id among those
// neighbours (Eq. 1 with ties to the lower id).  Processes the bricks listed
// for this level (items first, first + stride, ...); a brick that reached
// anything lists itself and its neighbours for L + 1.
__device__ void bfs_level(const BFSArgs &A, uint32_t L, const uint32_t *off, uint32_t tag, uint32_t first,
                          uint32_t stride) {
  const int t = threadIdx.x;
  const uint32_t count = off[kSub];
  const uint32_t *list_in = (L & 1) ? A.list1 : A.list0;
  uint32_t *list_out = (L & 1) ? A.list0 : A.list1;
  uint32_t *out_cnt = A.cnt + ((L + 1) % 3) * kSub;
  const uint32_t *fin = A.fr + (size_t)((L - 1) & 1) * A.bg.nbricks * kRows;
  uint32_t *fout = A.fr + (size_t)(L & 1) * A.bg.nbricks * kRows;
  const int ly = t & 15, lz = t >> 4;
  const int64_t sy = A.g.nx, sz = (int64_t)A.g.nx * A.g.ny;
  for (uint32_t item = first; item < count; item += stride) {
    // item -> (sub-list, position) by bisection over the sub-list offsets
    uint32_t lo = 0, hi = kSub;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (off[mid] <= item)
        lo = mid;
      else
        hi = mid;
    }
    const uint32_t b = list_in[(size_t)lo * A.bg.nbricks + (item - off[lo])];
    const int bx = (int)(b % A.bg.nbx), by = (int)((b / A.bg.nbx) % A.bg.nby), bz = (int)(b / ((uint32_t)A.bg.nbx * A.bg.nby));
    const int64_t rb = (int64_t)b * kRows;
    const int64_t bsy = A.bg.nbx, bsz = (int64_t)A.bg.nbx * A.bg.nby;
    const uint32_t F = fin[rb + t];
    const uint32_t vrow = A.vis[rb + t];
    const uint32_t fym = ly > 0 ? fin[rb + t - 1] : (by > 0 ? fin[(b - bsy) * kRows + t + 15] : 0u);
    const uint32_t fyp = ly < BY - 1 ? fin[rb + t + 1] : (by < A.bg.nby - 1 ? fin[(b + bsy) * kRows + t - 15] : 0u);
    const uint32_t fzm = lz > 0 ? fin[rb + t - 16] : (bz > 0 ? fin[(b - bsz) * kRows + t + 240] : 0u);
    const uint32_t fzp = lz < BZ - 1 ? fin[rb + t + 16] : (bz < A.bg.nbz - 1 ? fin[(b + bsz) * kRows + t - 240] : 0u);
    const uint32_t xin_m = bx > 0 ? (fin[(b - 1) * kRows + t] >> 15) & 1u : 0u;
    const uint32_t xin_p = bx < A.bg.nbx - 1 ? fin[(b + 1) * kRows + t] & 1u : 0u;
    const uint32_t sxm = (F << 1) | xin_m, sxp = (F >> 1) | (xin_p << 15);
    uint32_t nw = (sxm | sxp | fym | fyp | fzm | fzp) & ~vrow & 0xFFFFu;
    if (nw) {
      const uint32_t e0 = A.eq[(rb + t) * 3], e1 = A.eq[(rb + t) * 3 + 1], e2 = A.eq[(rb + t) * 3 + 2];
      const uint32_t fxm = sxm & e0 & 0xFFFFu, fxp = sxp & (e0 >> 16);
      const uint32_t gym = fym & e1, gyp = fyp & (e1 >> 16);
      const uint32_t gzm = fzm & e2, gzp = fzp & (e2 >> 16);
      nw &= fxm | fxp | gym | gyp | gzm | gzp;
      const int64_t base = brick_row_base(A.g, bx * BX, by * BY + ly, bz * BZ + lz);
      // ids of the new voxels, four at a time: all loads of a group are in
      // flight before its stores, so a row does not wait once per voxel
      uint32_t bits = nw;
      while (bits) {
        int xs[4];
        uint32_t idv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          xs[j] = bits ? __ffs(bits) - 1 : -1;
          bits &= bits - 1;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          uint32_t id = kNone;
          const int x = xs[j];
          if (x >= 0) {
            const int64_t v = base + x;
            if ((fxm >> x) & 1u) id = min(id, A.cell[v - 1]);
            if ((fxp >> x) & 1u) id = min(id, A.cell[v + 1]);
            if ((gym >> x) & 1u) id = min(id, A.cell[v - sy]);
            if ((gyp >> x) & 1u) id = min(id, A.cell[v + sy]);
            if ((gzm >> x) & 1u) id = min(id, A.cell[v - sz]);
            if ((gzp >> x) & 1u) id = min(id, A.cell[v + sz]);
          }
          idv[j] = id;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (xs[j] >= 0) A.cell[base + xs[j]] = idv[j];
      }
      if (nw) A.vis[rb + t] = vrow | nw;
    }
    fout[rb + t] = nw;
    if (__syncthreads_or(nw != 0) && t < kWave) queue_around(A, bx, by, bz, tag, list_out, out_cnt, b % kSub, 0x7Fu);
  }
}

// One BFS level per launch.  Workgroup 0 clears the list counter of level
// L + 2 (level L + 1 appends to it), so launches may be enqueued past the
// last level: they find an empty list and return.
__global__ __launch_bounds__(kVTThreads) void k_bfs_level(BFSArgs A, uint32_t L) {
  __shared__ uint32_t off[kSub + 1];
  const int t = threadIdx.x;
  if (t < kWave) {
    // exclusive prefix of the sub-list counts of level L
    const uint32_t c = t < kSub ? A.cnt[(L % 3) * kSub + t] : 0u;
    uint32_t inc = c;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t v = __shfl_up(inc, o, kWave);
      if (t >= o) inc += v;
    }
    if (t < kSub) off[t] = inc - c;
    if (t == kSub - 1) off[kSub] = inc;
    if (blockIdx.x == 0 && t < kSub) A.cnt[((L + 2) % 3) * kSub + t] = 0;  // level L + 1 lists into them
  }
  __syncthreads();
  if (blockIdx.x == 0 && t == 0) A.hist[L % kHistLen] = off[kSub];
  if (off[kSub] == 0) return;
  bfs_level(A, L, off, L + 1, blockIdx.x, gridDim.x);
}

// ----------------------------------------------------------------------------
// update

struct Sums {
  unsigned long long *M, *Sx, *Sy, *Sz;
};

// One workgroup per 64x8x8 tile; each wave takes rows of the tile with one
// lane per voxel (coalesced loads).  A segmented scan over the lanes sums
// (w, w x) over each run of equal cell id; the last lane of a run adds the
// run into an LDS hash table keyed by cell id, and the table is flushed with
// one set of global atomics per distinct cell in the tile.  Along a row y
// and z are fixed, so S_y = M y and S_z = M z per run.
constexpr int TX = 64, TY = 8, TZ = 8;
constexpr int kTabCap = 512;

__global__ __launch_bounds__(256) void k_centroid(const uint32_t *__restrict__ cell, const uint16_t *__restrict__ w,
                                                  Geom g, uint32_t S, Sums sums) {
  __shared__ uint32_t tkey[kTabCap];
  __shared__ unsigned long long tM[kTabCap], tX[kTabCap], tY[kTabCap], tZ[kTabCap];
  const int t = threadIdx.x, lane = lane_id(), wid = t / kWave;
  const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + TY - 1) / TY, ntz = (g.nz + TZ - 1) / TZ;
  const int64_t ntiles = (int64_t)ntx * nty * ntz;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    for (int i = t; i < kTabCap; i += 256) {
      tkey[i] = kNone;
      tM[i] = tX[i] = tY[i] = tZ[i] = 0ull;
    }
    __syncthreads();
    const int tx = (int)(tile % ntx), ty = (int)((tile / ntx) % nty), tz = (int)(tile / ((int64_t)ntx * nty));
    const int x = tx * TX + lane;
    for (int r = wid; r < TY * TZ; r += 256 / kWave) {
      const int y = ty * TY + (r & 7), z = tz * TZ + (r >> 3);
      if (y >= g.ny || z >= g.nz) continue;  // uniform across the wave
      const bool in = x < g.nx;
      const int64_t v = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
      const uint32_t c = in ? cell[v] : kNone;
      const uint32_t wv = in ? (w ? (uint32_t)w[v] : 1u) : 0u;
      // segmented inclusive scan over runs of equal c
      const uint32_t cl = __shfl_up(c, 1, kWave), cr = __shfl_down(c, 1, kWave);
      const bool head = lane == 0 || cl != c;
      const bool tail = lane == kWave - 1 || cr != c;
      uint32_t m = wv;
      uint64_t sx = (uint64_t)wv * (uint64_t)x;
      bool seg = head;
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t mo = __shfl_up(m, d, kWave);
        const uint64_t so = __shfl_up(sx, d, kWave);
        const bool fo = __shfl_up(seg ? 1 : 0, d, kWave) != 0;
        if (lane >= d && !seg) {
          m += mo;
          sx += so;
          seg = fo;
        }
      }
      if (tail && c < S && m) {
        const int sl = lds_slot<kTabCap>(tkey, c);
        if (sl >= 0) {
          atomicAdd(&tM[sl], (unsigned long long)m);
          atomicAdd(&tX[sl], (unsigned long long)sx);
          atomicAdd(&tY[sl], (unsigned long long)m * (uint64_t)y);
          atomicAdd(&tZ[sl], (unsigned long long)m * (uint64_t)z);
        } else {
          atomicAdd(&sums.M[c], (unsigned long long)m);
          atomicAdd(&sums.Sx[c], (unsigned long long)sx);
          atomicAdd(&sums.Sy[c], (unsigned long long)m * (uint64_t)y);
          atomicAdd(&sums.Sz[c], (unsigned long long)m * (uint64_t)z);
        }
      }
    }
    __syncthreads();
    for (int i = t; i < kTabCap; i += 256) {
      const uint32_t c = tkey[i];
      if (c != kNone && tM[i]) {
        atomicAdd(&sums.M[c], tM[i]);
        atomicAdd(&sums.Sx[c], tX[i]);
        atomicAdd(&sums.Sy[c], tY[i]);
        atomicAdd(&sums.Sz[c], tZ[i]);
      }
    }
    __syncthreads();
  }
}

struct U128 {
  uint64_t hi, lo;
};
__device__ __forceinline__ U128 sq64(uint64_t a) { return U128{__umul64hi(a, a), a * a}; }
__device__ __forceinline__ U128 add128(U128 a, U128 b) {
  uint64_t lo = a.lo + b.lo;
  return U128{a.hi + b.hi + (lo < a.lo ? 1ull : 0ull), lo};
}
__device__ __forceinline__ bool lt128(U128 a, U128 b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
__device__ __forceinline__ U128 shl2(U128 a) { return U128{(a.hi << 2) | (a.lo >> 62), a.lo << 2}; }
__device__ __forceinline__ uint64_t absdiff(uint64_t a, uint64_t b) { return a > b ? a - b : b - a; }

__device__ __forceinline__ uint64_t round_half_down(uint64_t S, uint64_t M) { return (2 * S + M - 1) / (2 * M); }

__device__ __forceinline__ double move_len(uint32_t a, uint32_t b, Geom g) {
  int64_t ax = a % (uint32_t)g.nx, ar = a / (uint32_t)g.nx, ay = ar % (uint32_t)g.ny, az = ar / (uint32_t)g.ny;
  int64_t bx = b % (uint32_t)g.nx, br = b / (uint32_t)g.nx, by = br % (uint32_t)g.ny, bz = br / (uint32_t)g.ny;
  double dx = (double)(ax - bx), dy = (double)(ay - by), dz = (double)(az - bz);
  return sqrt(dx * dx + dy * dy + dz * dz);
}

__global__ void k_snap(const uint32_t *__restrict__ cell, Geom g, uint32_t S, Sums sums, uint32_t *sites, double *ds,
                       uint32_t *fb_list, uint32_t *fb_cnt) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  uint64_t M = sums.M[s];
  uint32_t old = sites[s];
  if (M == 0) {
    if (ds) ds[s] = 0.0;
    return;
  }
  uint64_t qx = round_half_down(sums.Sx[s], M), qy = round_half_down(sums.Sy[s], M), qz = round_half_down(sums.Sz[s], M);
  uint32_t q = (uint32_t)(qx + (uint64_t)g.nx * (qy + (uint64_t)g.ny * qz));
  if (cell[q] == s) {
    sites[s] = q;
    if (ds) ds[s] = move_len(old, q, g);
  } else {
    uint32_t pos = atomicAdd(fb_cnt, 1u);
    fb_list[pos] = s;
  }
}

// Exact nearest in-cell voxel by growing cubes; one workgroup per site.
__global__ __launch_bounds__(256) void k_snap_fallback(const uint32_t *__restrict__ cell, Geom g, Sums sums,
                                                       uint32_t *sites, double *ds, const uint32_t *fb_list,
                                                       const uint32_t *fb_cnt) {
  __shared__ uint64_t r_hi[256], r_lo[256];
  __shared__ uint32_t r_v[256];
  const int t = threadIdx.x;
  const uint32_t count = *fb_cnt;
  for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) {
    const uint32_t s = fb_list[item];
    const uint64_t M = sums.M[s];
    const uint64_t Sa[3] = {sums.Sx[s], sums.Sy[s], sums.Sz[s]};
    const int64_t q[3] = {(int64_t)round_half_down(Sa[0], M), (int64_t)round_half_down(Sa[1], M),
                          (int64_t)round_half_down(Sa[2], M)};
    const int64_t ext[3] = {g.nx, g.ny, g.nz};
    U128 best{~0ull, ~0ull};
    uint32_t bestv = kNone;
    for (int64_t r = 1;; r *= 2) {
      int64_t lo[3], hi[3], len[3];
      bool whole = true;
      for (int a = 0; a < 3; ++a) {
        lo[a] = q[a] - r < 0 ? 0 : q[a] - r;
        hi[a] = q[a] + r > ext[a] - 1 ? ext[a] - 1 : q[a] + r;
        len[a] = hi[a] - lo[a] + 1;
        whole = whole && lo[a] == 0 && hi[a] == ext[a] - 1;
      }
      const int64_t vol = len[0] * len[1] * len[2];
      for (int64_t i = t; i < vol; i += 256) {
        int64_t cx = lo[0] + i % len[0];
        int64_t rr = i / len[0];
        int64_t cy = lo[1] + rr % len[1];
        int64_t cz = lo[2] + rr / len[1];
        int64_t v = cx + (int64_t)g.nx * (cy + (int64_t)g.ny * cz);
        if (cell[v] != s) continue;
        U128 D = sq64(absdiff(M * (uint64_t)cx, Sa[0]));
        D = add128(D, sq64(absdiff(M * (uint64_t)cy, Sa[1])));
        D = add128(D, sq64(absdiff(M * (uint64_t)cz, Sa[2])));
        if (lt128(D, best) || (D.hi == best.hi && D.lo == best.lo && (uint32_t)v < bestv)) {
          best = D;
          bestv = (uint32_t)v;
        }
      }
      r_hi[t] = best.hi;
      r_lo[t] = best.lo;
      r_v[t] = bestv;
      __syncthreads();
      for (int o = 128; o > 0; o >>= 1) {
        if (t < o) {
          U128 a{r_hi[t], r_lo[t]}, b{r_hi[t + o], r_lo[t + o]};
          uint32_t av = r_v[t], bv = r_v[t + o];
          if (lt128(b, a) || (b.hi == a.hi && b.lo == a.lo && bv < av)) {
            r_hi[t] = b.hi;
            r_lo[t] = b.lo;
            r_v[t] = bv;
          }
        }
        __syncthreads();
      }
      best = U128{r_hi[0], r_lo[0]};
      bestv = r_v[0];
      __syncthreads();
      bool done = whole;
      if (!done && bestv != kNone) {
        U128 bound = sq64(M * (uint64_t)(2 * r + 1));
        done = lt128(shl2(best), bound);
      }
      if (done) break;
    }
    if (t == 0) {
      uint32_t old = sites[s];
      if (bestv != kNone) {
        sites[s] = bestv;
        if (ds) ds[s] = move_len(old, bestv, g);
      } else if (ds) {
        ds[s] = 0.0;
      }
    }
    __syncthreads();
  }
}

// Mean of ds[0..S) in a fixed order: 256 contiguous chunks summed by 256
// workgroups, then the chunk sums in order by one workgroup.
constexpr int kMeanParts = 256;
__global__ __launch_bounds__(256) void k_mean_ds_part(const double *ds, uint32_t S, double *part) {
  __shared__ double red[256];
  const uint32_t chunk = (S + kMeanParts - 1) / kMeanParts;
  const uint32_t b0 = blockIdx.x * chunk;
  const uint32_t b1 = b0 + chunk < S ? b0 + chunk : S;
  double acc = 0.0;
  for (uint32_t i = b0 + threadIdx.x; i < b1; i += 256) acc += ds[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_mean_ds(const double *part, uint32_t S, double *out) {
  __shared__ double red[256];
  red[threadIdx.x] = part[threadIdx.x];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = S ? red[0] / (double)S : 0.0;
}

__global__ void k_init_sites(const uint32_t *__restrict__ seeds, uint32_t S, const uint32_t *__restrict__ comp, Geom g,
                             uint32_t *sites, uint32_t *site_comp, uint32_t *err) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  uint32_t v = seeds[s];
  if ((int64_t)v >= g.n) {
    atomicOr(err, 1u);
    v = 0;  // keep later kernels in bounds; the call reports EINVAL
  }
  sites[s] = v;
  site_comp[s] = comp[v];
}

// ----------------------------------------------------------------------------
// host side

struct CvtWork {
  uint32_t *eq, *fr, *vis;
  uint32_t *queued, *list_a, *list_b, *cnt;  // cnt[3][kSub] list counters, then error bits
  uint32_t *fb_list, *fb_cnt, *err;
  uint32_t *hist;
  unsigned long long *sums;  // 4 x S
  double *ds, *mean, *mean_part;
};

VTGrid vt_grid(const Geom &g) {
  VTGrid bg;
  bg.nbx = (g.nx + BX - 1) / BX;
  bg.nby = (g.ny + BY - 1) / BY;
  bg.nbz = (g.nz + BZ - 1) / BZ;
  bg.nbricks = (int64_t)bg.nbx * bg.nby * bg.nbz;
  return bg;
}

template <class A>
void cvt_layout(A &a, const Geom &g, uint32_t S, int32_t iters, CvtWork *W) {
  VTGrid bg = vt_grid(g);
  int64_t nb = bg.nbricks;
  size_t s1 = S ? S : 1;
  auto eq = a.template take<uint32_t>(nb * kRows * 3);
  auto fr = a.template take<uint32_t>(2 * nb * kRows);
  auto vis = a.template take<uint32_t>(nb * kRows);
  auto queued = a.template take<uint32_t>(nb);
  auto la = a.template take<uint32_t>((size_t)kSub * nb);
  auto lb = a.template take<uint32_t>((size_t)kSub * nb);
  auto cnt = a.template take<uint32_t>(3 * kSub + 1);  // list counters, then error bits
  auto fbl = a.template take<uint32_t>(s1);
  auto fbc = a.template take<uint32_t>(4);
  auto sums = a.template take<unsigned long long>(4 * s1);
  auto ds = a.template take<double>(s1);
  auto mean = a.template take<double>(iters > 0 ? iters : 1);
  auto mpart = a.template take<double>(kMeanParts);
  auto hist = a.template take<uint32_t>(kHistLen);
  if (W) {
    W->eq = eq;
    W->fr = fr;
    W->vis = vis;
    W->queued = queued;
    W->list_a = la;
    W->list_b = lb;
    W->cnt = cnt;
    W->err = cnt + 3 * kSub;
    W->fb_list = fbl;
    W->fb_cnt = fbc;
    W->sums = sums;
    W->ds = ds;
    W->mean = mean;
    W->mean_part = mpart;
    W->hist = hist;
  }
}

struct SizerT : Sizer {
  template <class T>
  T *take(size_t c) {
    Sizer::take<T>(c);
    return nullptr;
  }
};

size_t cvt_workspace(const Geom &g, uint32_t S, int32_t iters) {
  SizerT z;
  cvt_layout(z, g, S, iters, nullptr);
  return z.off + 256;
}

int32_t carve_cvt(void *d_work, size_t bytes, const Geom &g, uint32_t S, int32_t iters, CvtWork &W) {
  Carve cv(d_work, bytes);
  cvt_layout(cv, g, S, iters, &W);
  return cv.ok ? LSRVT_OK : LSRVT_EWORKSPACE;
}

// Driver state of one Lloyd run: the active-brick counts per level of the
// previous pass, which size the launches of the next one.
struct VTState {
  std::vector<uint32_t> prev;
};

// Benchmark timing of the level kernel: while enabled, an event pair on the
// launch stream around every batch of level launches; read back by
// lsrvt_timing_read.
struct KernelTimer {
  std::mutex mu;
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending, pool;
  double ms = 0.0;
  uint64_t launches = 0;
  uint64_t passes = 0;
  int64_t voxels_per_pass = 0;
};
KernelTimer &timer() {
  static KernelTimer t;
  return t;
}

int32_t timed_begin(hipStream_t s, std::pair<hipEvent_t, hipEvent_t> &ev) {
  KernelTimer &T = timer();
  std::lock_guard<std::mutex> lk(T.mu);
  if (T.pool.empty()) {
    hipEvent_t a, b;
    LSRVT_HIP(hipEventCreate(&a));
    LSRVT_HIP(hipEventCreate(&b));
    T.pool.push_back({a, b});
  }
  ev = T.pool.back();
  T.pool.pop_back();
  LSRVT_HIP(hipEventRecord(ev.first, s));
  return LSRVT_OK;
}

int32_t timed_end(hipStream_t s, const std::pair<hipEvent_t, hipEvent_t> &ev, uint64_t launches) {
  KernelTimer &T = timer();
  LSRVT_HIP(hipEventRecord(ev.second, s));
  std::lock_guard<std::mutex> lk(T.mu);
  T.pending.push_back(ev);
  T.launches += launches;
  return LSRVT_OK;
}

// Voxels never reached (components without a site) get LSRVT_NONE.
__global__ __launch_bounds__(kVTThreads) void k_vt_unreached(const uint32_t *__restrict__ vis, Geom g, VTGrid bg,
                                                             uint32_t *__restrict__ cell) {
  const int t = threadIdx.x, ly = t & 15, lz = t >> 4;
  for (int64_t b = blockIdx.x; b < bg.nbricks; b += gridDim.x) {
    const int bx = (int)(b % bg.nbx), by = (int)((b / bg.nbx) % bg.nby), bz = (int)(b / ((int64_t)bg.nbx * bg.nby));
    const int x0 = bx * BX, y = by * BY + ly, z = bz * BZ + lz;
    if (y >= g.ny || z >= g.nz) continue;
    const int w = g.nx - x0 < BX ? g.nx - x0 : BX;
    uint32_t miss = ~vis[b * kRows + t] & ((1u << w) - 1u);
    const int64_t base = brick_row_base(g, x0, y, z);
    while (miss) {
      const int x = __ffs(miss) - 1;
      miss &= miss - 1;
      cell[base + x] = kNone;
    }
  }
}

__global__ void k_sites_clear(const uint32_t *__restrict__ sites, uint32_t S, int64_t n, uint32_t *cell) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S && (int64_t)sites[s] < n) cell[sites[s]] = kNone;
}

unsigned vt_grid_cap(const VTGrid &bg) { return (unsigned)(bg.nbricks < 65535 ? bg.nbricks : 65535); }

int32_t vt_prepare(const uint8_t *band, const Geom &g, CvtWork &W, hipStream_t s) {
  VTGrid bg = vt_grid(g);
  const int64_t slots = bg.nbricks * kRows * BX;
  const unsigned grid = (unsigned)std::min<int64_t>((slots + kVTThreads - 1) / kVTThreads, 65535);
  hipLaunchKernelGGL(k_vt_eq, dim3(grid), dim3(kVTThreads), 0, s, band, g, bg, W.eq);
  LSRVT_LAUNCHED();
  return LSRVT_OK;
}

// One restricted Voronoi pass: level 0 at the sites, then one launch per BFS
// level over the bricks the front passes through, until a level reaches
// nothing.
// One restricted Voronoi pass: level 0 at the sites, then launches of the
// level kernel, enqueued in batches sized by the previous pass (sites move
// little between passes) until the device reports an empty level.
int32_t run_vt(const Geom &g, const uint32_t *sites, uint32_t S, uint32_t *cell, CvtWork &W, VTState &st,
               hipStream_t s) {
  VTGrid bg = vt_grid(g);
  int32_t rc;
  if ((rc = fill<uint32_t>(W.fr, 2 * bg.nbricks * kRows, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(W.vis, bg.nbricks * kRows, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(W.queued, bg.nbricks, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(W.cnt, 3 * kSub, 0u, s))) return rc;
  BFSArgs A;
  A.g = g;
  A.bg = bg;
  A.eq = W.eq;
  A.fr = W.fr;
  A.vis = W.vis;
  A.cell = cell;
  A.queued = W.queued;
  A.cnt = W.cnt;
  A.hist = W.hist;
  A.err = W.err;
  A.list0 = W.list_a;
  A.list1 = W.list_b;  // level 1 reads list1
  if (S) {
    hipLaunchKernelGGL(k_sites_clear, dim3((S + 255) / 256), dim3(256), 0, s, sites, S, g.n, cell);
    hipLaunchKernelGGL(k_bfs_init, dim3((S + 255) / 256), dim3(256), 0, s, sites, S, A, 1u);
    LSRVT_LAUNCHED();
  }
  const int64_t max_level = g.n + 2;
  const unsigned cap = vt_grid_cap(bg);
  uint32_t L = 0;  // levels enqueued
  int batch = st.prev.empty() ? 16 : (int)st.prev.size() + 4;
  bool more = S != 0;
  std::vector<uint32_t> c(3 * kSub + 1, 0);
  while (more) {
    // one event pair around a batch of back-to-back level launches (while
    // timing is on): the launches of a batch run without gaps
    const bool timed = timer().on;
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (timed && (rc = timed_begin(s, ev))) return rc;
    for (int i = 0; i < batch; ++i) {
      ++L;
      unsigned grid = cap;
      if (L - 1 < st.prev.size()) {
        const uint32_t p = st.prev[L - 1];
        grid = (unsigned)std::min<uint64_t>(cap, (uint64_t)p + p / 4 + 64);
      } else if (!st.prev.empty()) {
        grid = 64;  // most likely past the last level
      }
      hipLaunchKernelGGL(k_bfs_level, dim3(grid), dim3(kVTThreads), 0, s, A, L);
      LSRVT_LAUNCHED();
    }
    if (timed && (rc = timed_end(s, ev, (uint64_t)batch))) return rc;
    LSRVT_HIP(hipMemcpyAsync(c.data(), W.cnt, sizeof(uint32_t) * c.size(), hipMemcpyDeviceToHost, s));
    LSRVT_HIP(hipStreamSynchronize(s));
    const uint32_t e = c[3 * kSub];
    if (e & 1u) return LSRVT_EINVAL;
    if (e) return LSRVT_EDEVICE;
    more = false;  // bricks listed for the next level?
    for (int j = 0; j < kSub; ++j) more = more || c[((L + 1) % 3) * kSub + j] != 0;
    if ((int64_t)L > max_level) return LSRVT_EDEVICE;
    batch = 8;
  }
  const uint32_t launched = L;
  // the brick counts of levels 1 .. L size the next pass (trailing empty levels dropped)
  const uint32_t nl = std::min<uint32_t>(L + 1, kHistLen);
  std::vector<uint32_t> h(nl, 0);
  if (nl > 1) {
    LSRVT_HIP(hipMemcpyAsync(h.data(), W.hist, sizeof(uint32_t) * nl, hipMemcpyDeviceToHost, s));
    LSRVT_HIP(hipStreamSynchronize(s));
  }
  uint32_t levels = 0;
  while (levels + 1 < nl && h[levels + 1]) ++levels;
  st.prev.assign(h.begin() + 1, h.begin() + 1 + levels);
  hipLaunchKernelGGL(k_vt_unreached, dim3(cap), dim3(kVTThreads), 0, s, W.vis, g, bg, cell);
  LSRVT_LAUNCHED();
  if (timer().on) {
    std::lock_guard<std::mutex> lk(timer().mu);
    timer().passes += 1;
    timer().voxels_per_pass = g.n;
  }
  static const bool debug_levels = getenv("LSRVT_DEBUG_LEVELS") != nullptr;
  if (debug_levels) {
    fprintf(stderr, "[lsrvt] vt levels=%u launches=%u active bricks:", levels, launched);
    for (uint32_t l = 1; l <= levels; ++l) fprintf(stderr, " %u", h[l]);
    fprintf(stderr, "\n");
  }
  return LSRVT_OK;
}

// Errors a run reported on the device (synchronises).
int32_t vt_errors(CvtWork &W, hipStream_t s) {
  uint32_t e = 0;
  LSRVT_HIP(hipMemcpyAsync(&e, W.err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  LSRVT_HIP(hipStreamSynchronize(s));
  if (e & 1u) return LSRVT_EINVAL;
  if (e) return LSRVT_EDEVICE;
  return LSRVT_OK;
}

int32_t run_update(const uint32_t *cell, const Geom &g, const uint16_t *w, uint32_t *sites, uint32_t S, double *ds,
                   CvtWork &W, hipStream_t s) {
  if (S == 0) return LSRVT_OK;
  int32_t rc;
  if ((rc = fill<unsigned long long>(W.sums, 4 * (int64_t)S, 0ull, s))) return rc;
  if ((rc = fill<uint32_t>(W.fb_cnt, 1, 0u, s))) return rc;
  Sums sm{W.sums, W.sums + S, W.sums + 2 * (size_t)S, W.sums + 3 * (size_t)S};
  const int64_t ntiles = (int64_t)((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY) * ((g.nz + TZ - 1) / TZ);
  hipLaunchKernelGGL(k_centroid, dim3((unsigned)(ntiles < 65535 ? ntiles : 65535)), dim3(256), 0, s, cell, w, g, S, sm);
  hipLaunchKernelGGL(k_snap, dim3((S + 255) / 256), dim3(256), 0, s, cell, g, S, sm, sites, ds, W.fb_list, W.fb_cnt);
  hipLaunchKernelGGL(k_snap_fallback, dim3(S < 1024 ? S : 1024), dim3(256), 0, s, cell, g, sm, sites, ds, W.fb_list,
                     W.fb_cnt);
  LSRVT_LAUNCHED();
  return LSRVT_OK;
}

int32_t begin(CvtWork &W, const Geom &g, hipStream_t s) {
  int32_t rc;
  VTGrid bg = vt_grid(g);
  if ((rc = fill<uint32_t>(W.queued, bg.nbricks, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(W.cnt, 3 * kSub + 1, 0u, s))) return rc;
  return LSRVT_OK;
}

}  // namespace

}  // namespace lsrvt

using namespace lsrvt;

extern "C" size_t lsrvt_cvt_workspace(lsrvt_dims dims, uint32_t n_sites, int32_t iters) {
  Geom g;
  if (make_geom(dims, g)) return 0;
  return cvt_workspace(g, n_sites, iters < 0 ? 0 : iters);
}

extern "C" int32_t lsrvt_vt(const uint8_t *d_band, lsrvt_dims dims, const uint32_t *d_sites, uint32_t n_sites,
                            uint32_t *d_cell, void *d_work, size_t work_bytes, void *stream) {
  Geom g;
  int32_t rc = make_geom(dims, g);
  if (rc) return rc;
  if (!d_band || !d_cell || (n_sites && !d_sites)) return LSRVT_EINVAL;
  if ((rc = check_work(d_work, work_bytes, cvt_workspace(g, n_sites, 0)))) return rc;
  CvtWork W;
  if ((rc = carve_cvt(d_work, work_bytes, g, n_sites, 0, W))) return rc;
  hipStream_t s = as_stream(stream);
  if ((rc = begin(W, g, s))) return rc;
  if ((rc = vt_prepare(d_band, g, W, s))) return rc;
  VTState st;
  if ((rc = run_vt(g, d_sites, n_sites, d_cell, W, st, s))) return rc;
  return vt_errors(W, s);
}

extern "C" int32_t lsrvt_update(const uint32_t *d_cell, lsrvt_dims dims, const uint16_t *d_weights, uint32_t *d_sites,
                                uint32_t n_sites, double *d_ds, void *d_work, size_t work_bytes, void *stream) {
  Geom g;
  int32_t rc = make_geom(dims, g);
  if (rc) return rc;
  if (!d_cell || (n_sites && !d_sites)) return LSRVT_EINVAL;
  if ((rc = check_work(d_work, work_bytes, cvt_workspace(g, n_sites, 0)))) return rc;
  CvtWork W;
  if ((rc = carve_cvt(d_work, work_bytes, g, n_sites, 0, W))) return rc;
  return run_update(d_cell, g, d_weights, d_sites, n_sites, d_ds, W, as_stream(stream));
}

extern "C" int32_t lsrvt_cvt(const uint8_t *d_band, const uint32_t *d_comp, lsrvt_dims dims, const uint32_t *d_seeds,
                             uint32_t n_sites, const uint16_t *d_weights, int32_t iters, uint32_t *d_cell,
                             uint32_t *d_sites, uint32_t *d_site_comp, double *h_mean_ds, void *d_work,
                             size_t work_bytes, void *stream) {
  Geom g;
  int32_t rc = make_geom(dims, g);
  if (rc) return rc;
  if (iters < 0) return LSRVT_EINVAL;
  if (!d_band || !d_comp || !d_cell || (n_sites && (!d_seeds || !d_sites || !d_site_comp))) return LSRVT_EINVAL;
  if ((rc = check_work(d_work, work_bytes, cvt_workspace(g, n_sites, iters)))) return rc;
  CvtWork W;
  if ((rc = carve_cvt(d_work, work_bytes, g, n_sites, iters, W))) return rc;
  hipStream_t s = as_stream(stream);
  if ((rc = begin(W, g, s))) return rc;
  if (n_sites) {
    hipLaunchKernelGGL(k_init_sites, dim3((n_sites + 255) / 256), dim3(256), 0, s, d_seeds, n_sites, d_comp, g, d_sites,
                       d_site_comp, W.err);
    LSRVT_LAUNCHED();
  }
  if ((rc = vt_prepare(d_band, g, W, s))) return rc;
  VTState st;
  for (int32_t t = 0; t <= iters; ++t) {
    if ((rc = run_vt(g, d_sites, n_sites, d_cell, W, st, s))) return rc;
    if (t == iters) break;
    if ((rc = run_update(d_cell, g, d_weights, d_sites, n_sites, W.ds, W, s))) return rc;
    hipLaunchKernelGGL(k_mean_ds_part, dim3(kMeanParts), dim3(256), 0, s, W.ds, n_sites, W.mean_part);
    hipLaunchKernelGGL(k_mean_ds, dim3(1), dim3(256), 0, s, W.mean_part, n_sites, W.mean + t);
    LSRVT_LAUNCHED();
  }
  if (h_mean_ds && iters > 0) {
    LSRVT_HIP(hipMemcpyAsync(h_mean_ds, W.mean, sizeof(double) * iters, hipMemcpyDeviceToHost, s));
  }
  return vt_errors(W, s);
}

extern "C" int32_t lsrvt_timing_enable(int32_t enable) {
  KernelTimer &T = timer();
  std::lock_guard<std::mutex> lk(T.mu);
  T.on = enable != 0;
  return LSRVT_OK;
}

extern "C" int32_t lsrvt_timing_read(double *ms, uint64_t *launches, uint64_t *passes, int64_t *voxels_per_pass) {
  KernelTimer &T = timer();
  std::lock_guard<std::mutex> lk(T.mu);
  for (auto &ev : T.pending) {
    LSRVT_HIP(hipEventSynchronize(ev.second));
    float dt = 0.0f;
    LSRVT_HIP(hipEventElapsedTime(&dt, ev.first, ev.second));
    T.ms += dt;
    T.pool.push_back(ev);
  }
  T.pending.clear();
  if (ms) *ms = T.ms;
  if (launches) *launches = T.launches;
  if (passes) *passes = T.passes;
  if (voxels_per_pass) *voxels_per_pass = T.voxels_per_pass;
  T.ms = 0.0;
  T.launches = 0;
  T.passes = 0;
  return LSRVT_OK;
}
