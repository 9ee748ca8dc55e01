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
// search keeps 16-bit masks in global memory: the same-band edges in each
// direction (built once per call, since bands do not change), the voxels
// reached so far and the frontier of the last two levels, plus the
// frontier's brick faces packed into a few words for the neighbours to read.
// A level launch has one wave per brick; a brick works only if it was marked
// for the level (a brick that reached anything marks itself and its six
// neighbours for the next one, with plain stores of the level number).
// Frontier words of bricks that reached nothing at a level are stale, but
// only hold voxels whose neighbours were all reached one level after them,
// so they are masked off by the reached mask, and a voxel that is new at
// some level has no such stale neighbour.  Each voxel is written once per
// pass.
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
#include <cmath>
#include <mutex>
#include <utility>
#include <vector>

#include "common.h"

namespace lsrvt {

namespace {

constexpr int BX = 16, BY = 16, BZ = 16;
constexpr int kRows = BY * BZ;  // a brick is 256 rows of 16 voxels along x
constexpr int kVTThreads = 256;
constexpr int kHistLen = 8192;  // per-level record of which levels reached anything

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
  uint16_t *fr;        // [2][nbricks][256] voxels reached at the level of that parity
  uint16_t *vis;       // [nbricks][256] voxels reached so far
  unsigned long long *xf;  // [2][nbricks][8] x = 0 face (words 0..3), x = 15 face (4..7) of the frontier;
                           // bit t of word k is row (t & 15) + 16 (4 (t >> 4) + k)
  uint16_t *yf;        // [2][nbricks][32] y = 0 face rows (0..15), y = 15 face rows (16..31) of the frontier, by z
  uint32_t *cell;      // [nbricks][4096] site id of every reached voxel, brick-major (x + 16 y + 256 z in the brick)
  uint32_t *dist;      // [nbricks][4096] level at which each voxel was reached (its hop distance), brick-major
  uint32_t *act;       // [2][nbricks]: act[L & 1][b] == L when brick b takes part in level L
  uint32_t *alive;     // [3]: alive[L % 3] != 0 when some brick takes part in level L
  uint32_t *hist;      // [kHistLen] alive flag of every level
  uint32_t *err;
  // incremental passes only
  uint16_t *inv;       // [nbricks][256] voxels whose site moved in the last update
  uint32_t *bnd;       // [nbricks][4096] kept voxels next to an invalid one: dist << 12 | x + 16 row
  uint32_t *bcnt;      // [nbricks] entries of bnd
  uint32_t *wake;      // [nbricks] next level at which the brick injects kept voxels (NONE: none)
  unsigned long long *dbg;  // diagnostics (LSRVT_DEBUG_LEVELS only): brick visits, candidates, ...
};

// Entries of the kept-voxel lists hold the level in 20 bits; a pass whose
// lists would need more runs as a full pass.
constexpr uint32_t kMaxBndLevel = (1u << 20) - 1;

__device__ __forceinline__ int64_t brick_row_base(const Geom &g, int x0, int y, int z) {
  return x0 + (int64_t)g.nx * (y + (int64_t)g.ny * z);
}

// Marks brick (bx, by, bz) and its six face neighbours for level L (plain
// stores: every writer stores the same tag).
__device__ __forceinline__ void mark_brick(const BFSArgs &A, int bx, int by, int bz, int k, uint32_t L) {
  const int qx = bx + (k == 1 ? -1 : k == 2 ? 1 : 0);
  const int qy = by + (k == 3 ? -1 : k == 4 ? 1 : 0);
  const int qz = bz + (k == 5 ? -1 : k == 6 ? 1 : 0);
  if (qx >= 0 && qy >= 0 && qz >= 0 && qx < A.bg.nbx && qy < A.bg.nby && qz < A.bg.nbz)
    A.act[(size_t)(L & 1) * A.bg.nbricks + (size_t)(qx + A.bg.nbx * (qy + A.bg.nby * qz))] = L;
}

// Same-band masks of every row toward its six neighbours (across brick faces
// too); voxels outside the volume have no edges.  One voxel per lane, so a
// wave covers four rows of a brick and the band reads are coalesced.  Bands
// do not change during a Lloyd loop, so this runs once per call.
__device__ __forceinline__ void d_vt_eq(const uint8_t *__restrict__ band, Geom g, VTGrid bg,
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
__global__ __launch_bounds__(kVTThreads) void k_vt_eq(const uint8_t *__restrict__ band, Geom g, VTGrid bg,
                                                      uint32_t *__restrict__ eq) { d_vt_eq(band, g, bg, eq); }


struct BrickPos {
  uint32_t b, row, lx;
  int bx, by, bz;
  size_t bi;  // brick-major index: b * 4096 + lx + 16 * row
};

__device__ __forceinline__ BrickPos brick_pos(const BFSArgs &A, uint32_t v) {
  const uint32_t x = v % (uint32_t)A.g.nx, r = v / (uint32_t)A.g.nx;
  const uint32_t y = r % (uint32_t)A.g.ny, z = r / (uint32_t)A.g.ny;
  BrickPos p;
  p.bx = (int)(x / BX);
  p.by = (int)(y / BY);
  p.bz = (int)(z / BZ);
  p.b = (uint32_t)p.bx + (uint32_t)A.bg.nbx * ((uint32_t)p.by + (uint32_t)A.bg.nby * (uint32_t)p.bz);
  p.row = (y % BY) + BY * (z % BZ);
  p.lx = x % BX;
  p.bi = (size_t)p.b * (kRows * BX) + p.lx + BX * p.row;
  return p;
}

// Bit of voxel (row, lx) of brick b in a 16-bit row array, read through the
// 32-bit word that holds it.
__device__ __forceinline__ bool row_bit(const uint16_t *rows, const BrickPos &p) {
  return (rows[(size_t)p.b * kRows + p.row] >> p.lx) & 1u;
}

__device__ __forceinline__ void or_row_bit(uint16_t *rows, const BrickPos &p) {
  const size_t w = ((size_t)p.b * kRows + p.row) >> 1;
  atomicOr(reinterpret_cast<uint32_t *>(rows) + w, (1u << p.lx) << ((p.row & 1u) * 16u));
}

// Puts a voxel into the frontier of level 0 (rows and packed faces) and
// marks its brick and the six neighbours for level 1.
__device__ void frontier0(const BFSArgs &A, const BrickPos &p) {
  or_row_bit(A.fr, p);
  const uint32_t ly = p.row & 15u, lz = p.row >> 4;
  if (p.lx == 0 || p.lx == BX - 1) {
    const uint32_t lane = ly + 16u * (lz >> 2), k = lz & 3u;
    atomicOr(&A.xf[(size_t)p.b * 8 + (p.lx ? 4 : 0) + k], 1ull << lane);
  }
  if (ly == 0 || ly == BY - 1) {
    const size_t yi = (size_t)p.b * 32 + (ly ? 16 : 0) + lz;
    atomicOr(reinterpret_cast<uint32_t *>(A.yf) + (yi >> 1), (1u << p.lx) << ((yi & 1u) * 16u));
  }
  // the brick, and the face neighbours whose shared face the voxel lies on
  const uint32_t lz2 = p.row >> 4, ly2 = p.row & 15u;
  const bool on[7] = {true, p.lx == 0, p.lx == BX - 1, ly2 == 0, ly2 == BY - 1, lz2 == 0, lz2 == BZ - 1};
#pragma unroll
  for (int k = 0; k < 7; ++k)
    if (on[k]) mark_brick(A, p.bx, p.by, p.bz, k, 1u);
  A.alive[1] = 1u;
}

// Level 0: every site reaches its own voxel; co-located sites keep the lowest id.
__global__ void k_bfs_init(const uint32_t *__restrict__ sites, uint32_t S, BFSArgs A) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  uint32_t v = sites[s];
  if ((int64_t)v >= A.g.n) {
    atomicOr(A.err, 1u);
    return;
  }
  const BrickPos p = brick_pos(A, v);
  atomicMin(&A.cell[p.bi], s);
  A.dist[p.bi] = 0u;
  or_row_bit(A.vis, p);
  frontier0(A, p);
}

// ----------------------------------------------------------------------------
// Incremental passes.  After an update only the sites that moved can change
// the regions.  A voxel whose site did not move keeps a key (distance, id)
// that is still the best over the sites that did not move, so the new key is
// the better of that one and the best over the moved sites; voxels whose site
// moved ("invalid") know neither.  The pass is the same level-synchronous
// search, restricted: its frontier at level L holds the voxels changed at
// level L - 1 and the kept voxels of distance L - 1 that touch an invalid
// voxel ("boundary", injected from per-brick lists at their level).  An
// invalid voxel reached at level L takes the smallest id of its frontier
// neighbours, as in a full pass: every neighbour at distance L - 1 is in the
// frontier (it changed, or it was kept and touches this invalid voxel).  A
// kept voxel reached at level L takes (L, id) only when that key is smaller
// than its own: a kept neighbour at distance L - 1 offers a key it already
// beats, so leaving such neighbours out of the frontier changes nothing.  A
// kept voxel that changes joins the frontier, so changes spread as far as
// they reach, and the result is the full pass's.

// Invalid rows: voxels whose site moved.  One voxel per lane, ballots per row
// (the slot index is the brick-major index of the cells).
__global__ __launch_bounds__(kVTThreads) void k_inc_reset(const uint32_t *__restrict__ cellb,
                                                          const uint8_t *__restrict__ moved, Geom g, VTGrid bg,
                                                          uint16_t *__restrict__ inv) {
  const int64_t slots = bg.nbricks * kRows * BX;
  const int lane = lane_id();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i - lane < slots;
       i += (int64_t)gridDim.x * blockDim.x) {
    bool p = false;
    const int64_t row = i >> 4;
    if (i < slots) {
      const int64_t b = row / kRows;
      const int t = (int)(row % kRows);
      const int bx = (int)(b % bg.nbx), by = (int)((b / bg.nbx) % bg.nby), bz = (int)(b / ((int64_t)bg.nbx * bg.nby));
      const int x = bx * BX + (int)(i & 15), y = by * BY + (t & 15), z = bz * BZ + (t >> 4);
      if (x < g.nx && y < g.ny && z < g.nz) {
        const uint32_t c = cellb[i];
        p = c != kNone && moved[c] != 0;
      }
    }
    const uint64_t m = __ballot(p);
    if (i < slots && (lane & 15) == 0) inv[row] = (uint16_t)((m >> lane) & 0xFFFFu);
  }
}

// Level 0 of an incremental pass, step 1: a site voxel changes when it is
// invalid or holds a larger key than (0, s); such voxels are cleared and
// flagged as changed (every writer stores the same values).
__global__ void k_inc_site_a(const uint32_t *__restrict__ sites, uint32_t S, BFSArgs A) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const uint32_t v = sites[s];
  if ((int64_t)v >= A.g.n) {
    atomicOr(A.err, 1u);
    return;
  }
  const BrickPos p = brick_pos(A, v);
  if (row_bit(A.inv, p) || A.dist[p.bi] != 0u || A.cell[p.bi] > s) {
    A.cell[p.bi] = kNone;
    A.dist[p.bi] = 0u;
    or_row_bit(A.vis, p);
  }
}

// Step 2: every site on a changed voxel takes part in the minimum; changed
// site voxels form the frontier of level 0.
__global__ void k_inc_site_b(const uint32_t *__restrict__ sites, uint32_t S, BFSArgs A) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const uint32_t v = sites[s];
  if ((int64_t)v >= A.g.n) return;
  const BrickPos p = brick_pos(A, v);
  if (!row_bit(A.vis, p)) return;
  atomicMin(&A.cell[p.bi], s);
  frontier0(A, p);
}

constexpr int kLvlThreads = 64;  // one wave per brick
constexpr int kNewCap = 1024;    // new voxels per brick and level shared out through LDS

// Ids of the six face neighbours of new voxel (lx, row) of brick b, the
// sources among them flagged by a0..a5 (x-, x+, y-, y+, z-, z+; at least one
// is set), read from the brick-major cell array.  A source across a brick
// face lies in the neighbour brick (which exists: edges join voxels of the
// volume only).  All six loads are issued unconditionally so that they are in
// flight together; a direction that is not a source reads the first source
// again, which hits the line that load brings in.
__device__ __forceinline__ void gather6(const uint32_t *cell, size_t b, uint32_t lx, uint32_t row, size_t bsy,
                                        size_t bsz, uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3, uint32_t a4,
                                        uint32_t a5, uint32_t g[6]) {
  constexpr size_t kB = (size_t)kRows * BX;
  const uint32_t ly = row & 15u, lz = row >> 4;
  const size_t v = b * kB + lx + BX * row;
  const size_t n0 = lx > 0 ? v - 1 : (b - 1) * kB + 15 + BX * row;
  const size_t n1 = lx < 15 ? v + 1 : (b + 1) * kB + BX * row;
  const size_t n2 = ly > 0 ? v - 16 : (b - bsy) * kB + lx + 16 * 15 + 256 * lz;
  const size_t n3 = ly < 15 ? v + 16 : (b + bsy) * kB + lx + 256 * lz;
  const size_t n4 = lz > 0 ? v - 256 : (b - bsz) * kB + lx + 16 * ly + 256 * 15;
  const size_t n5 = lz < 15 ? v + 256 : (b + bsz) * kB + lx + 16 * ly;
  size_t f = a5 ? n5 : v;
  f = a4 ? n4 : f;
  f = a3 ? n3 : f;
  f = a2 ? n2 : f;
  f = a1 ? n1 : f;
  f = a0 ? n0 : f;
  g[0] = cell[a0 ? n0 : f];
  g[1] = cell[a1 ? n1 : f];
  g[2] = cell[a2 ? n2 : f];
  g[3] = cell[a3 ? n3 : f];
  g[4] = cell[a4 ? n4 : f];
  g[5] = cell[a5 ? n5 : f];
}

__device__ __forceinline__ uint32_t min_id6(const uint32_t m0, const uint32_t m1, const uint32_t m2, const uint32_t g[6]) {
  uint32_t id = (m0 & 1u) ? g[0] : kNone;
  id = min(id, ((m0 >> 16) & 1u) ? g[1] : kNone);
  id = min(id, (m1 & 1u) ? g[2] : kNone);
  id = min(id, ((m1 >> 16) & 1u) ? g[3] : kNone);
  id = min(id, (m2 & 1u) ? g[4] : kNone);
  id = min(id, ((m2 >> 16) & 1u) ? g[5] : kNone);
  return id;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = min(v, (uint32_t)__shfl_xor(v, o, kWave));
  return v;
}

// LDS of one level workgroup (one wave).
struct LvlLds {
  uint16_t lst[kNewCap];   // listed candidates: x | row << 4
  uint32_t dmp[3 * kRows]; // per row: source directions of its candidates
  uint32_t inv[kRows];     // incremental: invalid voxels of candidate rows
  uint32_t acc[kRows];     // incremental: candidates that took a new key
  uint32_t inj[kRows];     // incremental: kept voxels injected at this level
};

// Level L: a candidate is a voxel that has not changed yet in this pass and
// has a same-band face neighbour in the frontier of level L - 1; its key
// would be (L, smallest id among those neighbours).  In a full pass every
// voxel is invalid and every candidate takes its key (Eq. 1 with ties to the
// lower id).  In an incremental pass a kept candidate takes it only when it
// is smaller than its own (distance, id).  One wave per brick: lane t owns
// the four rows ly = t & 15, lz = 4 (t >> 4) + k (k = 0..3), so the y- and
// z-neighbour rows inside the brick come from other lanes' registers, and
// the rows beyond the brick's faces from the neighbours' packed face words;
// every load of the brick's masks is issued at once.  Candidates are listed
// in LDS and shared out one per lane, whatever row they are in.  The
// frontier the brick writes for level L holds its changed voxels and, in an
// incremental pass, its kept voxels of distance L that touch an invalid one;
// when it is not empty the brick marks itself and its six neighbours for
// level L + 1.
template <bool INC>
__device__ void bfs_brick(const BFSArgs &A, uint32_t L, uint32_t b, LvlLds &S) {
  const int t = threadIdx.x;
  const int ly = t & 15, g4 = (t >> 4) * 4;
  const size_t pin = (size_t)((L - 1) & 1), pout = (size_t)(L & 1);
  const size_t nbk = (size_t)A.bg.nbricks;
  const uint16_t *fin = A.fr + pin * nbk * kRows;
  uint16_t *fout = A.fr + pout * nbk * kRows;
  const unsigned long long *xin = A.xf + pin * nbk * 8;
  unsigned long long *xout = A.xf + pout * nbk * 8;
  const uint16_t *yin = A.yf + pin * nbk * 32;
  uint16_t *yout = A.yf + pout * nbk * 32;
  const int64_t bsy = A.bg.nbx, bsz = (int64_t)A.bg.nbx * A.bg.nby;
  const int lm1 = (t + kWave - 1) & (kWave - 1), lp1 = (t + 1) & (kWave - 1);
  const int lm16 = (t + kWave - 16) & (kWave - 1), lp16 = (t + 16) & (kWave - 1);
  const int bx = (int)(b % A.bg.nbx), by = (int)((b / A.bg.nbx) % A.bg.nby), bz = (int)(b / ((uint32_t)A.bg.nbx * A.bg.nby));
  const int64_t rb = (int64_t)b * kRows;
  const bool hym = ly == 0 && by > 0, hyp = ly == BY - 1 && by < A.bg.nby - 1;
  uint32_t F[4], V[4], I[4], XM[4], XP[4], YM[4], YP[4], E[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = ly + 16 * (g4 + k);
#pragma unroll
    for (int j = 0; j < 3; ++j) E[k][j] = A.eq[(rb + r) * 3 + j];
    F[k] = fin[rb + r];
    V[k] = A.vis[rb + r];
    I[k] = INC ? (uint32_t)A.inv[rb + r] : 0xFFFFu;
    const unsigned long long xm = bx > 0 ? xin[(size_t)(b - 1) * 8 + 4 + k] : 0ull;
    const unsigned long long xp = bx < A.bg.nbx - 1 ? xin[(size_t)(b + 1) * 8 + k] : 0ull;
    XM[k] = (uint32_t)(xm >> t) & 1u;
    XP[k] = (uint32_t)(xp >> t) & 1u;
    YM[k] = hym ? yin[(size_t)(b - bsy) * 32 + 16 + g4 + k] : 0u;
    YP[k] = hyp ? yin[(size_t)(b + bsy) * 32 + g4 + k] : 0u;
  }
  const uint32_t ZM = (g4 == 0 && bz > 0) ? fin[(b - bsz) * kRows + 240 + ly] : 0u;
  const uint32_t ZP = (g4 == 12 && bz < A.bg.nbz - 1) ? fin[(b + bsz) * kRows + ly] : 0u;
  const uint32_t zlo = __shfl(F[3], lm16, kWave), zhi = __shfl(F[0], lp16, kWave);
  uint32_t cand[4], c = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = ly + 16 * (g4 + k);
    const uint32_t up = __shfl(F[k], lm1, kWave), dn = __shfl(F[k], lp1, kWave);
    const uint32_t fym = ly > 0 ? up : YM[k];
    const uint32_t fyp = ly < BY - 1 ? dn : YP[k];
    const uint32_t fzm = k > 0 ? F[k - 1] : (g4 > 0 ? zlo : ZM);
    const uint32_t fzp = k < 3 ? F[k + 1] : (g4 < 12 ? zhi : ZP);
    const uint32_t sxm = (F[k] << 1) | XM[k];
    const uint32_t sxp = (F[k] >> 1) | (XP[k] << 15);
    // reached from each direction: frontier neighbour with a same-band edge
    const uint32_t d0 = sxm & E[k][0] & 0xFFFFu, d1 = sxp & (E[k][0] >> 16);
    const uint32_t d2 = fym & E[k][1] & 0xFFFFu, d3 = fyp & (E[k][1] >> 16);
    const uint32_t d4 = fzm & E[k][2] & 0xFFFFu, d5 = fzp & (E[k][2] >> 16);
    cand[k] = (d0 | d1 | d2 | d3 | d4 | d5) & ~V[k] & 0xFFFFu;
    if (cand[k]) {
      S.dmp[r] = d0 | (d1 << 16);
      S.dmp[kRows + r] = d2 | (d3 << 16);
      S.dmp[2 * kRows + r] = d4 | (d5 << 16);
      if (INC) S.inv[r] = I[k];
    }
    c += (uint32_t)__popc(cand[k]);
  }
  // kept voxels of distance L that touch an invalid voxel join the frontier
  uint32_t inj[4] = {0u, 0u, 0u, 0u};
  if (INC && __builtin_amdgcn_readfirstlane(A.wake[b]) == L) {
#pragma unroll
    for (int k = 0; k < 4; ++k) S.inj[ly + 16 * (g4 + k)] = 0u;
    __syncthreads();
    const uint32_t cnt = A.bcnt[b];
    const uint32_t *list = A.bnd + (size_t)b * (kRows * BX);
    uint32_t nxt = kNone;
    for (uint32_t i = t; i < cnt; i += kWave) {
      const uint32_t e = list[i], d = e >> 12;
      if (d == L)
        atomicOr(&S.inj[(e & 0xFFFu) >> 4], 1u << (e & 15u));
      else if (d > L)
        nxt = min(nxt, d);
    }
    nxt = wave_min_u32(nxt);
    if (t == 0) A.wake[b] = nxt;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) inj[k] = S.inj[ly + 16 * (g4 + k)] & ~V[k];
  }
  uint32_t inc = c;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t v = __shfl_up(inc, o, kWave);
    if (t >= o) inc += v;
  }
  const uint32_t total = __shfl(inc, kWave - 1, kWave);
  const size_t vb = (size_t)b * (kRows * BX);  // the brick's first cell (brick-major arrays)
  uint32_t nw[4] = {0u, 0u, 0u, 0u};
  if (A.dbg && t == 0) {
    atomicAdd(reinterpret_cast<uint32_t *>(A.dbg + 8) + (L % kHistLen), 1u);
    atomicAdd(&A.dbg[0], 1ull);
    atomicAdd(&A.dbg[1], (unsigned long long)total);
    if (total > (uint32_t)kNewCap) {
      atomicAdd(&A.dbg[2], 1ull);
      atomicAdd(&A.dbg[3], (unsigned long long)total);
    }
  }
  if (total > 0 && total <= (uint32_t)kNewCap) {
    uint32_t p = inc - c;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      uint32_t bits = cand[k];
      const uint32_t r = (uint32_t)(ly + 16 * (g4 + k));
      if (INC) S.acc[r] = 0u;
      while (bits) {
        const uint32_t x = (uint32_t)(__ffs(bits) - 1);
        bits &= bits - 1;
        S.lst[p++] = (uint16_t)(x | (r << 4));
      }
    }
    __syncthreads();
    // keys of the listed voxels, two per lane at a time
    for (uint32_t e = t; e < total; e += 2 * kWave) {
      size_t v[2];
      uint32_t g[2][6], m[2][3], ob[2], od[2], oc[2], ri[2], xi[2];
      bool have[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const uint32_t ee = e + (uint32_t)u * kWave;
        have[u] = ee < total;
        const uint32_t idx = S.lst[have[u] ? ee : 0u];
        const uint32_t r = idx >> 4, x = idx & 15u;
        ri[u] = r;
        xi[u] = x;
        v[u] = vb + x + BX * r;
        m[u][0] = S.dmp[r] >> x;
        m[u][1] = S.dmp[kRows + r] >> x;
        m[u][2] = S.dmp[2 * kRows + r] >> x;
        gather6(A.cell, b, x, r, (size_t)bsy, (size_t)bsz, m[u][0] & 1u, (m[u][0] >> 16) & 1u, m[u][1] & 1u,
                (m[u][1] >> 16) & 1u, m[u][2] & 1u, (m[u][2] >> 16) & 1u, g[u]);
        ob[u] = INC ? (S.inv[r] >> x) & 1u : 1u;
        od[u] = 0u;
        oc[u] = 0u;
        if (!ob[u]) {  // a kept voxel: its own key
          od[u] = A.dist[v[u]];
          oc[u] = A.cell[v[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const uint32_t id = min_id6(m[u][0], m[u][1], m[u][2], g[u]);
        const bool ok = ob[u] || L < od[u] || (L == od[u] && id < oc[u]);
        if (have[u] && ok) {
          A.cell[v[u]] = id;
          A.dist[v[u]] = L;
          if (INC) atomicOr(&S.acc[ri[u]], 1u << xi[u]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) nw[k] = INC ? S.acc[ly + 16 * (g4 + k)] : cand[k];
  } else if (total > 0) {
    // more candidates than the list holds: each lane takes its own rows
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      uint32_t bits = cand[k];
      const int r = ly + 16 * (g4 + k);
      const size_t base = vb + BX * (size_t)r;
      const uint32_t m0 = S.dmp[r], m1 = S.dmp[kRows + r], m2 = S.dmp[2 * kRows + r];
      while (bits) {
        const int x = __ffs(bits) - 1;
        bits &= bits - 1;
        const size_t v = base + x;
        uint32_t gg[6];
        gather6(A.cell, b, (uint32_t)x, (uint32_t)r, (size_t)bsy, (size_t)bsz, (m0 >> x) & 1u, (m0 >> (16 + x)) & 1u,
                (m1 >> x) & 1u, (m1 >> (16 + x)) & 1u, (m2 >> x) & 1u, (m2 >> (16 + x)) & 1u, gg);
        const uint32_t id = min_id6(m0 >> x, m1 >> x, m2 >> x, gg);
        bool ok = true;
        if (INC && !((I[k] >> x) & 1u)) {
          const uint32_t od = A.dist[v], oc = A.cell[v];
          ok = L < od || (L == od && id < oc);
        }
        if (ok) {
          A.cell[v] = id;
          A.dist[v] = L;
          nw[k] |= 1u << x;
        }
      }
    }
  }
  uint32_t out[4], any = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    out[k] = nw[k] | inj[k];
    any |= out[k];
  }
  if (A.dbg) {
    uint32_t na = 0, ni = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      na += (uint32_t)__popc(nw[k]);
      ni += (uint32_t)__popc(inj[k]);
    }
    na = wave_sum_u32(na);
    ni = wave_sum_u32(ni);
    if (t == 0) {
      atomicAdd(&A.dbg[4], (unsigned long long)na);
      atomicAdd(&A.dbg[5], (unsigned long long)ni);
    }
  }
  // nothing reached or injected: the frontier words of this parity stay
  // stale, which is harmless (see above)
  if (__ballot(any != 0u) == 0ull) return;
  // the brick works at level L + 1, and so does each face neighbour whose
  // shared face the frontier touches (only through it can the frontier
  // reach that neighbour's voxels)
  uint32_t fxm = 0, fxp = 0, fym = 0, fyp = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    fxm |= out[k] & 1u;
    fxp |= (out[k] >> 15) & 1u;
    fym |= ly == 0 ? out[k] : 0u;
    fyp |= ly == BY - 1 ? out[k] : 0u;
  }
  const uint32_t fzm = g4 == 0 ? out[0] : 0u, fzp = g4 == 12 ? out[3] : 0u;
  const uint32_t mk = 1u | (__ballot(fxm != 0u) ? 2u : 0u) | (__ballot(fxp != 0u) ? 4u : 0u) |
                      (__ballot(fym != 0u) ? 8u : 0u) | (__ballot(fyp != 0u) ? 16u : 0u) |
                      (__ballot(fzm != 0u) ? 32u : 0u) | (__ballot(fzp != 0u) ? 64u : 0u);
  if (t < 7 && ((mk >> t) & 1u)) mark_brick(A, bx, by, bz, t, L + 1);
  if (t == 0) A.alive[(L + 1) % 3] = 1u;
  // this level's frontier: rows, and the packed faces the neighbours read
  unsigned long long xw = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = ly + 16 * (g4 + k);
    if (nw[k]) A.vis[rb + r] = (uint16_t)(V[k] | nw[k]);
    fout[rb + r] = (uint16_t)out[k];
    const unsigned long long lo_k = __ballot(out[k] & 1u), hi_k = __ballot((out[k] >> 15) & 1u);
    if (t == k) xw = lo_k;
    if (t == 4 + k) xw = hi_k;
    if (ly == 0) yout[(size_t)b * 32 + g4 + k] = (uint16_t)out[k];
    if (ly == BY - 1) yout[(size_t)b * 32 + 16 + g4 + k] = (uint16_t)out[k];
  }
  if (t < 8) xout[(size_t)b * 8 + t] = xw;
  __syncthreads();  // the LDS lists and masks are reused by the next brick
}

// One BFS level per launch over the bricks marked for it (and, in an
// incremental pass, the bricks that inject kept voxels at this level).
// Workgroup 0 records whether level L is alive and clears the flag of level
// L + 2 (level L + 1 sets it), so launches may be enqueued past the last
// level: they find no marked brick and return.
template <bool INC>
__global__ __launch_bounds__(kLvlThreads) void k_bfs_level(BFSArgs A, uint32_t L) {
  __shared__ LvlLds S;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    A.hist[L % kHistLen] = A.alive[L % 3];
    A.alive[(L + 2) % 3] = 0u;
  }
  const uint32_t *act = A.act + (size_t)(L & 1) * A.bg.nbricks;
  // workgroups are dealt to the eight XCDs in turn (the grid is a multiple of
  // 8): XCD i % 8 takes the i-th eighth of the bricks, neighbours included
  const int64_t per = (A.bg.nbricks + 7) / 8;
  for (int64_t i = blockIdx.x; i < 8 * per; i += gridDim.x) {
    const int64_t b = (i & 7) * per + (i >> 3);
    if (b >= A.bg.nbricks) continue;
    bool go = __builtin_amdgcn_readfirstlane(act[b]) == L;
    if (INC && !go) go = __builtin_amdgcn_readfirstlane(A.wake[b]) == L;
    if (!go) continue;
    bfs_brick<INC>(A, L, (uint32_t)b, S);
  }
}

// Incremental pass set-up: per brick, the kept voxels (not invalid, not yet
// changed) with a same-band face neighbour that is invalid.  Those of
// distance 0 (sites) go into the frontier of level 0 at once; the others are
// listed as (distance << 12 | x + 16 row), and the brick's wake level is
// their smallest distance.  One wave per brick, rows as in the level kernel.
__global__ __launch_bounds__(kLvlThreads) void k_bnd_build(BFSArgs A) {
  __shared__ uint16_t lst[kRows * BX];
  __shared__ uint32_t cnt_s;
  const int t = threadIdx.x;
  const int ly = t & 15, g4 = (t >> 4) * 4;
  const int lm1 = (t + kWave - 1) & (kWave - 1), lp1 = (t + 1) & (kWave - 1);
  const int lm16 = (t + kWave - 16) & (kWave - 1), lp16 = (t + 16) & (kWave - 1);
  const int64_t bsy = A.bg.nbx, bsz = (int64_t)A.bg.nbx * A.bg.nby;
  for (int64_t b = blockIdx.x; b < A.bg.nbricks; b += gridDim.x) {
    const int bx = (int)(b % A.bg.nbx), by = (int)((b / A.bg.nbx) % A.bg.nby),
              bz = (int)(b / ((int64_t)A.bg.nbx * A.bg.nby));
    const int64_t rb = b * kRows;
    const bool hym = ly == 0 && by > 0, hyp = ly == BY - 1 && by < A.bg.nby - 1;
    uint32_t I[4], V[4], XM[4], XP[4], YM[4], YP[4], E[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = ly + 16 * (g4 + k);
#pragma unroll
      for (int j = 0; j < 3; ++j) E[k][j] = A.eq[(rb + r) * 3 + j];
      I[k] = A.inv[rb + r];
      V[k] = A.vis[rb + r];
      XM[k] = bx > 0 ? ((uint32_t)A.inv[(b - 1) * kRows + r] >> 15) & 1u : 0u;
      XP[k] = bx < A.bg.nbx - 1 ? (uint32_t)A.inv[(b + 1) * kRows + r] & 1u : 0u;
      YM[k] = hym ? A.inv[(b - bsy) * kRows + 15 + 16 * (g4 + k)] : 0u;
      YP[k] = hyp ? A.inv[(b + bsy) * kRows + 16 * (g4 + k)] : 0u;
    }
    const uint32_t ZM = (g4 == 0 && bz > 0) ? A.inv[(b - bsz) * kRows + 240 + ly] : 0u;
    const uint32_t ZP = (g4 == 12 && bz < A.bg.nbz - 1) ? A.inv[(b + bsz) * kRows + ly] : 0u;
    const uint32_t zlo = __shfl(I[3], lm16, kWave), zhi = __shfl(I[0], lp16, kWave);
    uint32_t bm[4], c = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t up = __shfl(I[k], lm1, kWave), dn = __shfl(I[k], lp1, kWave);
      const uint32_t fym = ly > 0 ? up : YM[k];
      const uint32_t fyp = ly < BY - 1 ? dn : YP[k];
      const uint32_t fzm = k > 0 ? I[k - 1] : (g4 > 0 ? zlo : ZM);
      const uint32_t fzp = k < 3 ? I[k + 1] : (g4 < 12 ? zhi : ZP);
      const uint32_t sxm = (I[k] << 1) | XM[k];
      const uint32_t sxp = (I[k] >> 1) | (XP[k] << 15);
      const uint32_t adj = (sxm & E[k][0] & 0xFFFFu) | (sxp & (E[k][0] >> 16)) | (fym & E[k][1] & 0xFFFFu) |
                           (fyp & (E[k][1] >> 16)) | (fzm & E[k][2] & 0xFFFFu) | (fzp & (E[k][2] >> 16));
      bm[k] = adj & ~I[k] & ~V[k] & 0xFFFFu;
      c += (uint32_t)__popc(bm[k]);
    }
    uint32_t inc = c;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t v = __shfl_up(inc, o, kWave);
      if (t >= o) inc += v;
    }
    const uint32_t total = __shfl(inc, kWave - 1, kWave);
    if (total == 0) {
      if (t == 0) {
        A.bcnt[b] = 0u;
        A.wake[b] = kNone;
      }
      continue;
    }
    uint32_t p = inc - c;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      uint32_t bits = bm[k];
      const uint32_t r = (uint32_t)(ly + 16 * (g4 + k));
      while (bits) {
        const uint32_t x = (uint32_t)(__ffs(bits) - 1);
        bits &= bits - 1;
        lst[p++] = (uint16_t)(x | (r << 4));
      }
    }
    if (t == 0) cnt_s = 0u;
    __syncthreads();
    const size_t vb = (size_t)b * (kRows * BX);
    uint32_t *list = A.bnd + (size_t)b * (kRows * BX);
    uint32_t nxt = kNone;
    for (uint32_t e = t; e < total; e += kWave) {
      const uint32_t idx = lst[e];
      const uint32_t r = idx >> 4, x = idx & 15u;
      const uint32_t d = A.dist[vb + x + BX * r];
      if (d == 0u) {
        BrickPos q;
        q.b = (uint32_t)b;
        q.row = r;
        q.lx = x;
        q.bx = bx;
        q.by = by;
        q.bz = bz;
        frontier0(A, q);
      } else if (d > kMaxBndLevel) {
        atomicOr(A.err, 4u);
      } else {
        list[atomicAdd(&cnt_s, 1u)] = (d << 12) | idx;
        nxt = min(nxt, d);
      }
    }
    nxt = wave_min_u32(nxt);
    __syncthreads();
    if (t == 0) {
      A.bcnt[b] = cnt_s;
      A.wake[b] = nxt;
    }
    __syncthreads();
  }
}

// Smallest wake level over all bricks (the next level at which some brick
// injects kept voxels), atomically into *out, which holds NONE beforehand.
__global__ __launch_bounds__(256) void k_wake_min(const uint32_t *__restrict__ wake, int64_t nb, uint32_t *out) {
  uint32_t m = kNone;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (int64_t)gridDim.x * blockDim.x)
    m = min(m, wake[i]);
  m = wave_min_u32(m);
  if (lane_id() == 0 && m != kNone) atomicMin(out, m);
}

// ----------------------------------------------------------------------------
// Brick relaxation engine (an alternative schedule for the same regions).
//
// The regions of Eq. 1 with ties to the lower id are the unique fixed point
// of key(v) = min(key(v), min over same-band face neighbours w of
// key(w) + (1, 0)), keys (distance, id) compared lexicographically and
// packed as distance << 32 | id, started from (0, s) at the sites and
// "unreached" elsewhere.  Any order of such relaxations that starts from
// keys that are lengths of real paths (upper bounds) and stops when nothing
// changes reaches that fixed point, so the result is the level search's, bit
// for bit.  Here a round is one launch over the bricks marked for it: a
// workgroup loads a brick's keys into LDS, takes the offers of the six face
// neighbours (their stored keys plus one hop), relaxes the brick to its own
// fixed point by line sweeps along x, y and z (forward and backward, with the
// same-band edge masks) until a sweep round changes nothing, stores the keys
// that changed, and marks for the next round each face neighbour whose shared
// face changed.  A brick reads its neighbours' keys while they may be
// written in the same round: every value it can see is a real path length,
// and a neighbour that lowers a face key after the read marks it again, so
// the rounds end exactly at the fixed point.  An incremental pass starts from
// the previous keys with the voxels of moved sites set to unreached.  That
// reset is done either by its own kernel (which marks the bricks that hold
// such voxels), or fused into the first round, which then works on every
// brick: each key it reads (the brick's own and the neighbours' faces) is
// taken as unreached when its site moved, unless it is the site's own new
// voxel, and it stores the whole brick.  Keys seen in the first round are
// thus always the reset ones, whichever bricks have been stored already.
//
// Keys come in two widths.  Wide keys are 64 bits, distance << 32 | id.
// Narrow keys are 32 bits, distance << b | id with b the bits the site ids
// need (at most 24 by default); one hop adds 1 << b with unsigned
// saturation, so a key that would pass 2^32 - 1 stays "unreached" (all
// ones), which is never an offer.  Every key of a voxel whose true
// distance is below D = 2^(32 - b) - 2 is then exact (its shortest path
// never saturates), and a voxel farther away has a voxel at distance
// exactly D on its shortest path.  So a round that stores a key of
// distance D or more flags the pass, and the host repeats the pass (and
// runs the rest of the call) with wide keys; a pass that ends unflagged
// has every distance below D and is exact.
constexpr int kBRThreads = 256;
constexpr int kBRRow = BX + 1;  // LDS row stride (keys): padding against bank conflicts
constexpr int kGraphRounds = 8;  // relaxation rounds per captured graph

struct BRArgs {
  Geom g;
  VTGrid bg;
  const uint32_t *eq;              // [nbricks][256][3] same-band edge masks (as the level search)
  void *key;                       // [nbricks][4096] brick-major keys (narrow or wide), all ones = unreached
  void *xface;                     // [nbricks][2][256] keys of the x = 0 and x = 15 voxels of every row
  uint32_t hop32;                  // narrow keys: one hop (1 << b)
  uint32_t idmask;                 // the id bits of a key (0xFFFFFFFF for wide keys)
  uint32_t lim32;                  // narrow keys: the smallest key whose distance is D (flagged when stored)
  uint32_t *mark;                  // [2][nbricks]: mark[r & 1][b] == r when brick b works in round r
  uint32_t *list;                  // [nbricks] bricks of the current round
  uint32_t *ctl;                   // [0] list length, [2] reset fused into round 1, [3] error bits
  const uint8_t *moved;            // the sites the last update moved (fused reset)
  const uint32_t *fsites;          // the sites' voxels (fused reset)
  uint32_t *rnd;                   // the current round (advanced on the device, so rounds replay from a graph)
  uint32_t *alive;                 // [3] round alive flags (by r % 3); shared by the jobs of a batch
  uint32_t *hist;                  // [kHistLen] bricks that worked in each round
  unsigned long long *dbg;         // diagnostics (LSRVT_DEBUG_LEVELS only): processings, sweep rounds
};

// The two key widths: unreached value, one hop, and key + hop, which stays
// unreached from unreached (a wide key tests for it, a narrow one
// saturates).
template <class KT>
struct BRKey;
template <>
struct BRKey<unsigned long long> {
  static constexpr unsigned long long inf = ~0ull;
  __device__ static unsigned long long hop(const BRArgs &) { return 1ull << 32; }
  __device__ static unsigned long long add(unsigned long long k, unsigned long long h) {
    return k == inf ? inf : k + h;
  }
};
template <>
struct BRKey<uint32_t> {
  static constexpr uint32_t inf = ~0u;
  __device__ static uint32_t hop(const BRArgs &A) { return A.hop32; }
  __device__ static uint32_t add(uint32_t k, uint32_t h) { return __builtin_elementwise_add_sat(k, h); }
};

// A key of the previous pass as the fused reset sees it at voxel v:
// unreached when its site moved, unless it is that site's new voxel
// (distance 0 at the site's voxel).
template <class KT>
__device__ __forceinline__ KT br_filter(const BRArgs &A, KT k, KT hop, uint32_t v) {
  if (k == BRKey<KT>::inf) return k;
  const uint32_t id = (uint32_t)k & A.idmask;
  if (!A.moved[id] || (k < hop && A.fsites[id] == v)) return k;
  return BRKey<KT>::inf;
}

// *p = min(*p, k) with the stored value taken through the fused reset's
// filter; returns whether k was stored.
template <class KT>
__device__ __forceinline__ bool br_cas_min(const BRArgs &A, KT *p, KT k, KT hop, uint32_t v) {
  KT old = __atomic_load_n(p, __ATOMIC_RELAXED);
  for (;;) {
    if (k >= br_filter<KT>(A, old, hop, v)) return false;
    const KT prev = atomicCAS(p, old, k);
    if (prev == old) return true;
    old = prev;
  }
}

__device__ __forceinline__ void br_mark(const BRArgs &A, int bx, int by, int bz, int k, uint32_t r) {
  const int qx = bx + (k == 1 ? -1 : k == 2 ? 1 : 0);
  const int qy = by + (k == 3 ? -1 : k == 4 ? 1 : 0);
  const int qz = bz + (k == 5 ? -1 : k == 6 ? 1 : 0);
  if (qx >= 0 && qy >= 0 && qz >= 0 && qx < A.bg.nbx && qy < A.bg.nby && qz < A.bg.nbz)
    A.mark[(size_t)(r & 1) * A.bg.nbricks + (size_t)(qx + A.bg.nbx * (qy + A.bg.nby * qz))] = r;
}

// Site keys of a pass: (0, s) wherever it is smaller than the stored key
// (every voxel of a full pass is unreached); a site voxel that changes
// marks its brick, and the face neighbours whose face it lies on, for round
// 1 (its packed x-face copy follows).
template <class KT>
__device__ __forceinline__ void d_br_sites(const uint32_t *__restrict__ sites, uint32_t S, BRArgs A) {
  KT *key = static_cast<KT *>(A.key), *xface = static_cast<KT *>(A.xface);
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const uint32_t v = sites[s];
  if ((int64_t)v >= A.g.n) {
    atomicOr(&A.ctl[3], 1u);
    return;
  }
  const uint32_t x = v % (uint32_t)A.g.nx, rr = v / (uint32_t)A.g.nx;
  const uint32_t y = rr % (uint32_t)A.g.ny, z = rr / (uint32_t)A.g.ny;
  const int bx = (int)(x / BX), by = (int)(y / BY), bz = (int)(z / BZ);
  const size_t b = (size_t)bx + (size_t)A.bg.nbx * ((size_t)by + (size_t)A.bg.nby * (size_t)bz);
  const uint32_t lx = x % BX, ly = y % BY, lz = z % BZ;
  const uint32_t row = ly + BY * lz;
  const KT k = (KT)s;
  if (A.ctl[2] == 0u) {
    const KT old = atomicMin(&key[b * (kRows * BX) + lx + BX * row], k);
    if (k >= old) return;
    if (lx == 0) atomicMin(&xface[b * 512 + row], k);
    if (lx == BX - 1) atomicMin(&xface[b * 512 + 256 + row], k);
  } else {  // previous keys, seen through the fused reset's filter
    const KT hop = BRKey<KT>::hop(A);
    if (!br_cas_min<KT>(A, &key[b * (kRows * BX) + lx + BX * row], k, hop, v)) return;
    if (lx == 0) br_cas_min<KT>(A, &xface[b * 512 + row], k, hop, v);
    if (lx == BX - 1) br_cas_min<KT>(A, &xface[b * 512 + 256 + row], k, hop, v);
  }
  const bool on[7] = {true, lx == 0, lx == BX - 1, ly == 0, ly == BY - 1, lz == 0, lz == BZ - 1};
#pragma unroll
  for (int q = 0; q < 7; ++q)
    if (on[q]) br_mark(A, bx, by, bz, q, 1u);
  A.alive[1] = 1u;
}
template <class KT>
__global__ void k_br_sites(const uint32_t *__restrict__ sites, uint32_t S, BRArgs A) { d_br_sites<KT>(sites, S, A); }


// Incremental pass set-up: voxels whose site moved become unreached (keys
// and packed faces), and their bricks are marked for round 1.  One thread
// per voxel slot (the slot index is the brick-major index).
template <class KT>
__device__ __forceinline__ void d_br_reset(const uint8_t *__restrict__ moved, BRArgs A) {
  constexpr KT kInf = BRKey<KT>::inf;
  KT *key = static_cast<KT *>(A.key), *xface = static_cast<KT *>(A.xface);
  const int64_t slots = A.bg.nbricks * kRows * BX;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int lane = lane_id();
  constexpr int kU = 8;  // slots per thread and step: their loads are issued together
  // A wave's 64 slots of a step lie in one brick (bricks are 4096 slots,
  // waves and the stride multiples of 64), so the loop bounds are the same
  // for the whole wave and one lane marks the brick.
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < slots; i0 += kU * stride) {
    KT k[kU];
    uint8_t mv[kU];
#pragma unroll
    for (int j = 0; j < kU; ++j) {
      const int64_t i = i0 + j * stride;
      k[j] = i < slots ? key[i] : kInf;
    }
#pragma unroll
    for (int j = 0; j < kU; ++j) mv[j] = k[j] != kInf ? moved[(uint32_t)k[j] & A.idmask] : (uint8_t)0;
#pragma unroll
    for (int j = 0; j < kU; ++j) {
      const int64_t i = i0 + j * stride;
      if (mv[j]) {
        key[i] = kInf;
        const int64_t b = i / (kRows * BX);
        const int loc = (int)(i % (kRows * BX));
        const int lx = loc & 15, row = loc >> 4;
        if (lx == 0) xface[b * 512 + row] = kInf;
        if (lx == BX - 1) xface[b * 512 + 256 + row] = kInf;
      }
      const uint64_t any = __ballot(mv[j] != 0);
      if (any && lane == __builtin_ctzll(any)) {
        A.mark[(size_t)1 * A.bg.nbricks + i / (kRows * BX)] = 1u;  // round 1 has parity 1
        A.alive[1] = 1u;
      }
    }
  }
}
// Sites the last update moved, counted into *out (zeroed before).
__global__ __launch_bounds__(256) void k_count_moved(const uint8_t *__restrict__ moved, uint32_t S, uint32_t *out) {
  uint32_t c = 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < S; i += gridDim.x * blockDim.x) c += moved[i] != 0;
  for (int o = kWave / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
  if (lane_id() == 0 && c) atomicAdd(out, c);
}

// Set-up of an incremental pass of lsrvt_cvt: with more than fuse_min
// sites moved (the count in ctl[1]; mode 0), or always (mode 2), the reset
// is fused into round 1 (ctl[2] set, every brick marked for round 1);
// otherwise (or always, mode 1) the voxels of moved sites are reset here.
template <class KT>
__global__ __launch_bounds__(256) void k_br_reset_or_fuse(const uint8_t *__restrict__ moved, BRArgs A,
                                                          uint32_t fuse_min, int32_t mode) {
  if (mode == 2 || (mode == 0 && A.ctl[1] > fuse_min)) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 == 0) {
      A.ctl[2] = 1u;
      A.alive[1] = 1u;
    }
    for (int64_t b = i0; b < A.bg.nbricks; b += (int64_t)gridDim.x * blockDim.x) A.mark[A.bg.nbricks + b] = 1u;
    return;
  }
  d_br_reset<KT>(moved, A);
}


// The bricks marked for round r, listed (one counter atomic per block on
// *cnt, zero before the launch).
__device__ __forceinline__ void d_br_list(BRArgs A, uint32_t r, uint32_t *cnt) {
  __shared__ uint32_t base_s;
  __shared__ uint32_t wcount[256 / kWave];
  const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
  if (blockIdx.x == 0 && t == 0) A.alive[(r + 2) % 3] = 0u;  // round r + 2 sets its flag during round r + 1
  const uint32_t *mk = A.mark + (size_t)(r & 1) * A.bg.nbricks;
  for (int64_t b0 = (int64_t)blockIdx.x * 256; b0 < A.bg.nbricks; b0 += (int64_t)gridDim.x * 256) {
    const int64_t b = b0 + t;
    const bool on = b < A.bg.nbricks && mk[b] == r;
    const uint64_t bal = __ballot(on);
    if (lane == 0) wcount[w] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (t == 0) {
      uint32_t tot = 0;
      for (int q = 0; q < 256 / kWave; ++q) tot += wcount[q];
      base_s = tot ? atomicAdd(cnt, tot) : 0u;
    }
    __syncthreads();
    uint32_t off = base_s;
    for (int q = 0; q < w; ++q) off += wcount[q];
    if (on) A.list[off + (uint32_t)__popcll(bal & lanemask_lt())] = (uint32_t)b;
    __syncthreads();
  }
}
// Rounds are replayed from a graph of kGraphRounds rounds: the round at
// position i of a replay is *rnd + 1 + i, and the graph's last kernel
// advances *rnd by kGraphRounds.  Round r's list length is counted in
// ctl[0] (odd r) or ctl[12] (even r); round r empties the counter of round
// r + 1 (nobody else touches it while round r runs).
__device__ __forceinline__ uint32_t *br_count(const BRArgs &A, uint32_t r) {
  return (r & 1u) ? &A.ctl[0] : &A.ctl[12];
}
__global__ void k_br_advance(BRArgs A) {
  if (threadIdx.x == 0) *A.rnd += (uint32_t)kGraphRounds;
}
__global__ __launch_bounds__(256) void k_br_list(BRArgs A, int32_t i) {
  const uint32_t r = *A.rnd + 1u + (uint32_t)i;
  d_br_list(A, r, br_count(A, r));
}


__device__ __forceinline__ int br_at(int lx, int row) { return row * kBRRow + lx; }

// One line of 16 voxels at K[base + i * st] relaxed forward and backward
// along its same-band edges (mask bit i: edge from voxel i to i - 1, bit
// 16 + i: edge to i + 1).  Returns the bits of the voxels whose key dropped;
// the line is written back only then.  The calling thread owns the line for
// the whole stage.  Branch-free: a missing edge turns the offer into all
// ones (never smaller).  The mask passes through an empty asm statement so
// that the per-voxel edge tests are made here, from one register, rather
// than hoisted out of the caller's sweep loop as lane masks (two scalar
// registers each, 90 for a thread's three lines).
template <class KT>
__device__ __forceinline__ uint32_t br_sweep(KT *K, int base, int st, uint32_t mask, KT hop) {
  using KO = BRKey<KT>;
  uint32_t nm = ~mask;
  asm volatile("" : "+v"(nm));
  // all ones when bit j of the mask is clear, else zero
  auto cut = [&](int j) { return (KT)(int64_t)((int32_t)(nm << (31 - j)) >> 31); };
  KT k[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) k[i] = K[base + i * st];
  // the changed bits are shifted in one at a time (no per-bit constants):
  // forward voxel i lands at bit 15 - i (reversed below), backward voxel i
  // at bit i
  uint32_t cf = 0, cb = 0;
#pragma unroll
  for (int i = 1; i < 16; ++i) {
    const KT o = KO::add(k[i - 1], hop) | cut(i);
    const bool lt = o < k[i];
    k[i] = lt ? o : k[i];
    cf = cf + cf + (uint32_t)lt;
  }
#pragma unroll
  for (int i = 14; i >= 0; --i) {
    const KT o = KO::add(k[i + 1], hop) | cut(16 + i);
    const bool lt = o < k[i];
    k[i] = lt ? o : k[i];
    cb = cb + cb + (uint32_t)lt;
  }
  const uint32_t c = (__builtin_bitreverse32(cf) >> 16) | cb;
  if (c) {
#pragma unroll
    for (int i = 0; i < 16; ++i) K[base + i * st] = k[i];
  }
  return c;
}

// One round over the listed bricks.  Thread t owns three lines of the
// brick for the whole processing: row t along x (ly, lz) = (t & 15, t >> 4),
// the y line (lx, lz) = (t & 15, t >> 4) and the z line (lx, ly) =
// (t & 15, t >> 4); their edge masks stay in registers.  LDS holds the
// keys (rows padded against bank conflicts), a changed bit per voxel and a
// dirty flag per line.
// LDS of one brick processing: the keys (rows padded against bank
// conflicts), the y and z edge masks by row (transposed into line masks),
// a changed bit per voxel, a dirty flag per line, the face flags.
template <class KT>
struct BRLds {
  KT K[kRows * kBRRow];
  uint32_t raw[2][kRows];
  uint32_t chg[kRows];                      // bit lx of row: the voxel's key changed in this processing
  uint8_t dx[kRows], dy[kRows], dz[kRows];  // lines to sweep along x (by row), y (lx, lz), z (lx, ly)
  uint32_t flags[8];
};

// One processing of brick b in round r (all threads of the workgroup).
template <class KT>
__device__ __forceinline__ void br_process(const BRArgs &A, int64_t b, uint32_t r, BRLds<KT> &L) {
  using KO = BRKey<KT>;
  constexpr KT kInf = KO::inf;
  const KT hop = KO::hop(A);
  KT *key = static_cast<KT *>(A.key), *xface = static_cast<KT *>(A.xface);
  KT *K = L.K;
  uint32_t(*raw)[kRows] = L.raw;
  uint32_t *chg = L.chg;
  uint8_t *dx = L.dx, *dy = L.dy, *dz = L.dz;
  uint32_t *flags = L.flags;
  // the thread index passes through an empty asm statement so that what is
  // derived from it (LDS and global offsets) is recomputed per processing
  // instead of being kept live across a round's processings
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  const int lo4 = t & 15, hi4 = t >> 4;
  const size_t kB = (size_t)kRows * BX;
  const int64_t bsy = A.bg.nbx, bsz = (int64_t)A.bg.nbx * A.bg.nby;
  {
    const int bx = (int)(b % A.bg.nbx), by = (int)((b / A.bg.nbx) % A.bg.nby),
              bz = (int)(b / ((int64_t)A.bg.nbx * A.bg.nby));
    const bool hxm = bx > 0, hxp = bx < A.bg.nbx - 1, hym = by > 0, hyp = by < A.bg.nby - 1, hzm = bz > 0,
               hzp = bz < A.bg.nbz - 1;
    // every global read of the processing, issued together: the brick's keys
    // (16 per thread, coalesced), its edge masks and the six faces of the
    // neighbours (a missing neighbour reads the brick itself, unused)
    KT kv[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) kv[i] = key[(size_t)b * kB + i * kBRThreads + t];
    const uint32_t *eq = A.eq + ((size_t)b * kRows + t) * 3;
    const uint32_t mx = eq[0], e1 = eq[1], e2 = eq[2];
    KT fxm = xface[(size_t)(hxm ? b - 1 : b) * 512 + 256 + t];
    KT fxp = xface[(size_t)(hxp ? b + 1 : b) * 512 + t];
    KT fym = key[(size_t)(hym ? b - bsy : b) * kB + lo4 + 16 * 15 + 256 * hi4];
    KT fyp = key[(size_t)(hyp ? b + bsy : b) * kB + lo4 + 256 * hi4];
    KT fzm = key[(size_t)(hzm ? b - bsz : b) * kB + lo4 + 16 * hi4 + 256 * 15];
    KT fzp = key[(size_t)(hzp ? b + bsz : b) * kB + lo4 + 16 * hi4];
    // first round of an incremental pass with the reset fused in
    const bool fuse = r == 1 && A.ctl[2] != 0u;
    if (fuse) {
      const uint32_t nx = (uint32_t)A.g.nx, nxy = (uint32_t)A.g.nx * (uint32_t)A.g.ny;
      const uint32_t x0 = (uint32_t)bx * BX, y0 = (uint32_t)by * BY, z0 = (uint32_t)bz * BZ;
      // thread t's voxel i is (x0 + lo4, y0 + hi4, z0 + i)
      const uint32_t v0 = x0 + lo4 + nx * (y0 + hi4) + nxy * z0;
#pragma unroll
      for (int i = 0; i < 16; ++i) kv[i] = br_filter<KT>(A, kv[i], hop, v0 + nxy * (uint32_t)i);
      // the face voxels' own coordinates (unused where the neighbour is missing)
      fxm = br_filter<KT>(A, fxm, hop, x0 - 1 + nx * (y0 + lo4) + nxy * (z0 + hi4));
      fxp = br_filter<KT>(A, fxp, hop, x0 + BX + nx * (y0 + lo4) + nxy * (z0 + hi4));
      fym = br_filter<KT>(A, fym, hop, x0 + lo4 + nx * (y0 - 1) + nxy * (z0 + hi4));
      fyp = br_filter<KT>(A, fyp, hop, x0 + lo4 + nx * (y0 + BY) + nxy * (z0 + hi4));
      fzm = br_filter<KT>(A, fzm, hop, x0 + lo4 + nx * (y0 + hi4) + nxy * (z0 - 1));
      fzp = br_filter<KT>(A, fzp, hop, x0 + lo4 + nx * (y0 + hi4) + nxy * (z0 + BZ));
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int loc = i * kBRThreads + t;
      K[br_at(loc & 15, loc >> 4)] = kv[i];
    }
    raw[0][t] = e1;
    raw[1][t] = e2;
    chg[t] = 0u;
    // In round 1 every line starts dirty (sites were set, keys reset or the
    // pass starts from nothing).  Later a brick's keys are a fixed point of
    // its own relaxation (its last processing ended at one, or the previous
    // pass's result is one), so only the lines through voxels that a
    // neighbour's offer lowered can change.
    dx[t] = dy[t] = dz[t] = r == 1 ? 1 : 0;
    if (t < 8) flags[t] = 0u;
    __syncthreads();
    // line masks of this thread's y line (lx, lz) and z line (lx, ly), in
    // the x rows' format (bit i: edge to i - 1, bit 16 + i: edge to i + 1)
    uint32_t my = 0, mz = 0;
#pragma unroll 2
    for (int i = 0; i < 16; ++i) {
      const uint32_t wy = raw[0][i + 16 * hi4], wz = raw[1][hi4 + 16 * i];
      my |= ((wy >> lo4) & 1u) << i | ((wy >> (16 + lo4)) & 1u) << (16 + i);
      mz |= ((wz >> lo4) & 1u) << i | ((wz >> (16 + lo4)) & 1u) << (16 + i);
    }
    // offers of the six face neighbours: their keys plus one hop
    {
      auto offer = [&](bool has, bool edge, KT h, int lx, int row) {
        const KT o = KO::add(h, hop);
        if (has && edge && h != kInf && atomicMin(&K[br_at(lx, row)], o) > o) {
          atomicOr(&chg[row], 1u << lx);
          dx[row] = 1;
          dy[lx + 16 * (row >> 4)] = 1;
          dz[lx + 16 * (row & 15)] = 1;
        }
      };
      offer(hxm, mx & 1u, fxm, 0, t);
      offer(hxp, (mx >> 31) & 1u, fxp, 15, t);
      offer(hym, my & 1u, fym, lo4, 16 * hi4);
      offer(hyp, (my >> 31) & 1u, fyp, lo4, 15 + 16 * hi4);
      offer(hzm, mz & 1u, fzm, lo4, hi4);
      offer(hzp, (mz >> 31) & 1u, fzp, lo4, hi4 + 16 * 15);
    }
    __syncthreads();
    // the brick's own fixed point: line sweeps along x, y and z.  A line is
    // swept (again) along its axis only after a voxel on it changed; the
    // loop ends when no line is dirty.
    uint32_t sweeps = 0;
    for (;;) {
      ++sweeps;
      if (dx[t]) {  // row t = (ly, lz)
        dx[t] = 0;
        uint32_t c = br_sweep<KT>(K, t * kBRRow, 1, mx, hop);
        chg[t] |= c;  // only this thread touches row t's word in this stage
        while (c) {
          const int x = __builtin_ctz(c);
          c &= c - 1;
          dy[x + 16 * hi4] = 1;
          dz[x + 16 * lo4] = 1;
        }
      }
      __syncthreads();
      if (dy[t]) {  // y line (lx, lz) = (lo4, hi4)
        dy[t] = 0;
        uint32_t c = br_sweep<KT>(K, 16 * kBRRow * hi4 + lo4, kBRRow, my, hop);
        while (c) {
          const int y = __builtin_ctz(c);
          c &= c - 1;
          atomicOr(&chg[y + 16 * hi4], 1u << lo4);
          dx[y + 16 * hi4] = 1;
          dz[lo4 + 16 * y] = 1;
        }
      }
      __syncthreads();
      if (dz[t]) {  // z line (lx, ly) = (lo4, hi4)
        dz[t] = 0;
        uint32_t c = br_sweep<KT>(K, hi4 * kBRRow + lo4, 16 * kBRRow, mz, hop);
        while (c) {
          const int z = __builtin_ctz(c);
          c &= c - 1;
          atomicOr(&chg[hi4 + 16 * z], 1u << lo4);
          dx[hi4 + 16 * z] = 1;
          dy[lo4 + 16 * z] = 1;
        }
      }
      __syncthreads();  // every dirty mark of the z stage is visible before the test
      if (!__syncthreads_or(dx[t] | dy[t] | dz[t])) break;
    }
    // Which neighbours work in round r + 1: a face voxel that changed, has a
    // same-band edge across the face and whose key plus one hop beats the
    // neighbour's voxel across it as read at the top.  Keys only decrease
    // within a pass, so a neighbour whose key already was no larger can never
    // take the offer.  Thread t checks the face voxels it offered to above.
    uint32_t fc = 0;
    {
      auto gain = [&](bool has, bool edge, int lx, int row, KT nbk) {
        if (!has || !edge || !((chg[row] >> lx) & 1u)) return false;
        const KT k = K[br_at(lx, row)];
        return KO::add(k, hop) < nbk;
      };
      fc |= gain(hxm, mx & 1u, 0, t, fxm) ? 2u : 0u;
      fc |= gain(hxp, (mx >> 31) & 1u, 15, t, fxp) ? 4u : 0u;
      fc |= gain(hym, my & 1u, lo4, 16 * hi4, fym) ? 8u : 0u;
      fc |= gain(hyp, (my >> 31) & 1u, lo4, 15 + 16 * hi4, fyp) ? 16u : 0u;
      fc |= gain(hzm, mz & 1u, lo4, hi4, fzm) ? 32u : 0u;
      fc |= gain(hzp, (mz >> 31) & 1u, lo4, hi4 + 16 * 15, fzp) ? 64u : 0u;
    }
    if (fc) atomicOr(&flags[0], fc);
    // store what changed.  The thread index is passed through an empty asm
    // statement so that the store addresses are recomputed here instead of
    // being kept live (in registers) from the loads at the top across the
    // sweeps.
    // A narrow key of distance D or more flags the pass (all ones is
    // unreached: stored by the fused reset, it flags nothing).
    int tt = t;
    asm volatile("" : "+v"(tt));
    bool far = false;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int loc = i * kBRThreads + tt;
      const int lx = loc & 15, row = loc >> 4;
      if (fuse || ((chg[row] >> lx) & 1u)) {
        const KT k = K[br_at(lx, row)];
        if (sizeof(KT) == 4) far |= (uint32_t)k >= A.lim32 && k != kInf;
        key[(size_t)b * kB + loc] = k;
        if (lx == 0) xface[(size_t)b * 512 + row] = k;
        if (lx == BX - 1) xface[(size_t)b * 512 + 256 + row] = k;
      }
    }
    if (sizeof(KT) == 4 && far) atomicOr(&A.ctl[3], 4u);
    if (A.dbg && t == 0) {
      atomicAdd(&A.dbg[0], 1ull);
      atomicAdd(&A.dbg[1], (unsigned long long)sweeps);
    }
    __syncthreads();
    // the neighbours that can gain work in round r + 1
    const uint32_t nb_exists = (hxm ? 2u : 0u) | (hxp ? 4u : 0u) | (hym ? 8u : 0u) | (hyp ? 16u : 0u) |
                               (hzm ? 32u : 0u) | (hzp ? 64u : 0u);
    const uint32_t f = flags[0] & nb_exists;
    if (t >= 1 && t < 7 && ((f >> t) & 1u)) br_mark(A, bx, by, bz, t, r + 1);
    if (t == 0 && f) A.alive[(r + 1) % 3] = 1u;
    __syncthreads();
  }
}

template <class KT>
__global__ __launch_bounds__(kBRThreads, sizeof(KT) == 4 ? 5 : 4) void k_br_round(BRArgs A, int32_t i) {
  __shared__ BRLds<KT> L;
  const uint32_t r = *A.rnd + 1u + (uint32_t)i;
  const uint32_t count = *br_count(A, r);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    A.hist[r % kHistLen] = count;  // bricks that work in round r
    *br_count(A, r + 1u) = 0u;
  }
  for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) br_process<KT>(A, A.list[item], r, L);
}


// ----------------------------------------------------------------------------
// update

struct Sums {
  unsigned long long *M, *Sx, *Sy, *Sz;
};

// The centroid sums of the update (Sec. 3.1: mass and mass-weighted
// position of every cell, exact uint64 integers, so their order does not
// matter) taken at the end of the Voronoi pass that produces the cells: the
// pass's last kernel holds every voxel's cell id once anyway, so the sums
// cost no second read of the cell array.  Partial sums go into an LDS
// table keyed by cell id (global atomics when the table is full), flushed
// with one set of global atomics per distinct cell of the workgroup's part.
// The level search's finish takes one workgroup per 16^3 brick: thread t
// takes voxel t, t + 256, ... of the brick, so the 16 lanes of each quarter
// wave hold one row along x, and a segmented scan over those 16 lanes (DPP
// row shifts) sums (w, w * (x - x0)) over every run of equal cell id, whose
// last lane adds it into the table.  The relaxation's finish keeps running
// sums per lane instead (d_br_finish_slabs).
struct Fuse {
  const uint16_t *w;  // weights (C order) or null for unit weights
  uint32_t S;
  Sums sums;          // zeroed before the pass
};

constexpr int kFinTab = 256;
struct FinTab {
  uint32_t tkey[kFinTab];
  unsigned long long tM[kFinTab], tX[kFinTab], tY[kFinTab], tZ[kFinTab];
};

__device__ __forceinline__ void fin_clear(FinTab &T) {
  for (int i = threadIdx.x; i < kFinTab; i += blockDim.x) {
    T.tkey[i] = kNone;
    T.tM[i] = T.tX[i] = T.tY[i] = T.tZ[i] = 0ull;
  }
}

// v moved right by CTRL's shift within each row of 16 lanes; 0 where the
// source lane lies outside the row.
template <int CTRL>
__device__ __forceinline__ uint32_t row_shift(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

// One voxel per lane, 16 lanes per row (lane & 15 = x - x0, every lane of
// the wave active): adds the runs of equal cell id of the wave's four rows
// into the table.  c = kNone for voxels outside the volume (weight 0).
__device__ __forceinline__ void fin_row_runs(FinTab &T, const Fuse &F, uint32_t c, uint32_t wv, uint32_t x0,
                                             uint32_t y, uint32_t z) {
  const uint32_t lx = threadIdx.x & 15;
  const uint32_t cl = (uint32_t)__builtin_amdgcn_update_dpp((int)kNone, (int)c, 0x111, 0xF, 0xF, false);  // row_shr:1
  const uint32_t cr = (uint32_t)__builtin_amdgcn_update_dpp((int)kNone, (int)c, 0x101, 0xF, 0xF, false);  // row_shl:1
  uint32_t m = wv, sx = wv * lx;  // sum of w * (x - x0) over a run: below 2^24
  uint32_t f = (lx == 0 || cl != c) ? 1u : 0u;  // a run starts within the lanes summed so far
#define LSRVT_SEG_STEP(CTRL)                                        \
  {                                                                 \
    const uint32_t mo = row_shift<CTRL>(m), so = row_shift<CTRL>(sx), fo = row_shift<CTRL>(f); \
    if (!f) {                                                       \
      m += mo;                                                      \
      sx += so;                                                     \
      f = fo;                                                       \
    }                                                               \
  }
  LSRVT_SEG_STEP(0x111)  // row_shr:1
  LSRVT_SEG_STEP(0x112)  // row_shr:2
  LSRVT_SEG_STEP(0x114)  // row_shr:4
  LSRVT_SEG_STEP(0x118)  // row_shr:8
#undef LSRVT_SEG_STEP
  const bool tail = lx == 15 || cr != c;
  if (tail && c < F.S && m) {
    const unsigned long long M = m, X = (unsigned long long)m * x0 + sx, Y = (unsigned long long)m * y,
                             Z = (unsigned long long)m * z;
    const int sl = lds_slot<kFinTab>(T.tkey, c);
    if (sl >= 0) {
      atomicAdd(&T.tM[sl], M);
      atomicAdd(&T.tX[sl], X);
      atomicAdd(&T.tY[sl], Y);
      atomicAdd(&T.tZ[sl], Z);
    } else {
      atomicAdd(&F.sums.M[c], M);
      atomicAdd(&F.sums.Sx[c], X);
      atomicAdd(&F.sums.Sy[c], Y);
      atomicAdd(&F.sums.Sz[c], Z);
    }
  }
}

// After the brick's rows (and a barrier): the table to global memory.  Ends
// with a barrier.
__device__ __forceinline__ void fin_flush(FinTab &T, const Fuse &F) {
  for (int i = threadIdx.x; i < kFinTab; i += blockDim.x) {
    const uint32_t c = T.tkey[i];
    if (c != kNone && T.tM[i]) {
      atomicAdd(&F.sums.M[c], T.tM[i]);
      atomicAdd(&F.sums.Sx[c], T.tX[i]);
      atomicAdd(&F.sums.Sy[c], T.tY[i]);
      atomicAdd(&F.sums.Sz[c], T.tZ[i]);
    }
  }
  __syncthreads();
}

// End of a relaxation pass: the keys to C-order cells (kNone where
// unreached) and, with SUMS, the centroid sums of the update that follows.
// One workgroup per slab of four x-adjacent bricks (64 x 16 x 16 voxels);
// lane l of every wave owns x = 64 sx + l, so a row's cells (256 B) and
// weights (128 B) are contiguous and each brick's 16 keys of the row are
// one 64 B run.  Wave w takes the slab's rows with z - z0 in [4w, 4w + 4),
// y fastest, eight rows per step with their loads issued together.  For
// the sums a lane keeps running totals (w, w (y - y0), w (z - z0)) of the
// cell it is in and adds them into the LDS table when its cell changes
// (w x = x times the mass, x being fixed per lane); the table goes to global
// memory once per slab.
constexpr int kFinRows = 8;
template <class KT, bool SUMS>
__device__ __forceinline__ void d_br_finish_slabs(const KT *__restrict__ key, Geom g, VTGrid bg, uint32_t idmask,
                                                  uint32_t *__restrict__ cell, const Fuse &F, FinTab *T) {
  const int t = threadIdx.x, lane = t & (kWave - 1), wv_id = t / kWave;
  const int nsx = (bg.nbx + 3) / 4;
  const int64_t nslabs = (int64_t)nsx * bg.nby * bg.nbz;
  for (int64_t sl = blockIdx.x; sl < nslabs; sl += gridDim.x) {
    const int sx = (int)(sl % nsx), by = (int)((sl / nsx) % bg.nby), bz = (int)(sl / ((int64_t)nsx * bg.nby));
    if constexpr (SUMS) {
      fin_clear(*T);
      __syncthreads();
    }
    const int bx = sx * 4 + (lane >> 4);
    const int x = bx * BX + (lane & 15);
    const bool has = bx < bg.nbx;  // the lane's brick exists
    const bool xin = x < g.nx;
    const int64_t b = (int64_t)(has ? bx : bg.nbx - 1) + (int64_t)bg.nbx * (by + (int64_t)bg.nby * bz);
    const KT *kb = key + (size_t)b * (kRows * BX) + (lane & 15);
    const int y0 = by * BY, z0 = bz * BZ;
    uint32_t cur = kNone, m = 0, sy = 0, sz = 0;  // the lane's running sums (below 2^26 over 64 rows)
    auto flush = [&]() {
      if (cur < F.S && m) {
        const unsigned long long M = m, X = (unsigned long long)m * (uint32_t)x,
                                 Y = (unsigned long long)m * (uint32_t)y0 + sy,
                                 Z = (unsigned long long)m * (uint32_t)z0 + sz;
        const int slot = lds_slot<kFinTab>(T->tkey, cur);
        if (slot >= 0) {
          atomicAdd(&T->tM[slot], M);
          atomicAdd(&T->tX[slot], X);
          atomicAdd(&T->tY[slot], Y);
          atomicAdd(&T->tZ[slot], Z);
        } else {
          atomicAdd(&F.sums.M[cur], M);
          atomicAdd(&F.sums.Sx[cur], X);
          atomicAdd(&F.sums.Sy[cur], Y);
          atomicAdd(&F.sums.Sz[cur], Z);
        }
      }
    };
    for (int j0 = 0; j0 < kRows / (kVTThreads / kWave); j0 += kFinRows) {
      KT k[kFinRows];
      uint32_t wt[kFinRows];
#pragma unroll
      for (int u = 0; u < kFinRows; ++u) {
        const int r = (kRows / (kVTThreads / kWave)) * wv_id + j0 + u;  // (ly, lz) = (r & 15, r >> 4)
        const bool rin = y0 + (r & 15) < g.ny && z0 + (r >> 4) < g.nz;
        k[u] = has && rin ? kb[r * BX] : BRKey<KT>::inf;
        if constexpr (SUMS) {
          const int64_t v = (int64_t)g.nx * ((y0 + (r & 15)) + (int64_t)g.ny * (z0 + (r >> 4))) + x;
          wt[u] = xin && rin ? (F.w ? (uint32_t)F.w[v] : 1u) : 0u;
        }
      }
#pragma unroll
      for (int u = 0; u < kFinRows; ++u) {
        const int r = (kRows / (kVTThreads / kWave)) * wv_id + j0 + u;
        const int ly = r & 15, lz = r >> 4;
        const bool in = xin && y0 + ly < g.ny && z0 + lz < g.nz;
        const uint32_t c = k[u] == BRKey<KT>::inf ? kNone : (uint32_t)k[u] & idmask;
        if (in) cell[(int64_t)g.nx * ((y0 + ly) + (int64_t)g.ny * (z0 + lz)) + x] = c;
        if constexpr (SUMS) {
          const uint32_t cc = in ? c : kNone;
          if (cc != cur) {
            flush();
            cur = cc;
            m = sy = sz = 0;
          }
          m += wt[u];
          sy += wt[u] * (uint32_t)ly;
          sz += wt[u] * (uint32_t)lz;
        }
      }
    }
    if constexpr (SUMS) {
      flush();
      __syncthreads();
      fin_flush(*T, F);
    }
  }
}

template <class KT>
__global__ __launch_bounds__(kVTThreads) void k_br_finish_sums(const KT *__restrict__ key, Geom g, VTGrid bg,
                                                               uint32_t idmask, uint32_t *__restrict__ cell, Fuse F) {
  __shared__ FinTab T;
  d_br_finish_slabs<KT, true>(key, g, bg, idmask, cell, F, &T);
}
template <class KT>
__global__ __launch_bounds__(kVTThreads) void k_br_finish(const KT *__restrict__ key, Geom g, VTGrid bg,
                                                          uint32_t idmask, uint32_t *__restrict__ cell) {
  d_br_finish_slabs<KT, false>(key, g, bg, idmask, cell, Fuse{}, nullptr);
}

// One workgroup per 64x8x8 tile; each wave takes rows of the tile with one
// lane per voxel (coalesced loads).  A segmented scan over the lanes sums
// (w, w x) over each run of equal cell id; the last lane of a run adds the
// run into an LDS hash table keyed by cell id, and the table is flushed with
// one set of global atomics per distinct cell in the tile.  Along a row y
// and z are fixed, so S_y = M y and S_z = M z per run.
constexpr int TX = 64, TY = 8, TZ = 8;
constexpr int kTabCap = 512;

__device__ __forceinline__ void d_centroid(const uint32_t *__restrict__ cell, const uint16_t *__restrict__ w,
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
__global__ __launch_bounds__(256) void k_centroid(const uint32_t *__restrict__ cell, const uint16_t *__restrict__ w,
                                                  Geom g, uint32_t S, Sums sums) { d_centroid(cell, w, g, S, sums); }


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

// moved[s] records whether site s moved (the next Voronoi pass is
// incremental over the moved sites).
__device__ __forceinline__ void d_snap(const uint32_t *__restrict__ cell, Geom g, uint32_t S, Sums sums, uint32_t *sites, double *ds,
                       uint8_t *moved, uint32_t *fb_list, uint32_t *fb_cnt) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  uint64_t M = sums.M[s];
  uint32_t old = sites[s];
  moved[s] = 0;
  if (M == 0) {
    if (ds) ds[s] = 0.0;
    return;
  }
  uint64_t qx = round_half_down(sums.Sx[s], M), qy = round_half_down(sums.Sy[s], M), qz = round_half_down(sums.Sz[s], M);
  uint32_t q = (uint32_t)(qx + (uint64_t)g.nx * (qy + (uint64_t)g.ny * qz));
  if (cell[q] == s) {
    sites[s] = q;
    moved[s] = q != old;
    if (ds) ds[s] = move_len(old, q, g);
  } else {
    uint32_t pos = atomicAdd(fb_cnt, 1u);
    fb_list[pos] = s;
  }
}
__global__ void k_snap(const uint32_t *__restrict__ cell, Geom g, uint32_t S, Sums sums, uint32_t *sites, double *ds,
                       uint8_t *moved, uint32_t *fb_list, uint32_t *fb_cnt) { d_snap(cell, g, S, sums, sites, ds, moved, fb_list, fb_cnt); }


// Exact nearest in-cell voxel by growing cubes; one workgroup per site.
__device__ __forceinline__ void d_snap_fallback(const uint32_t *__restrict__ cell, Geom g, Sums sums,
                                                       uint32_t *sites, double *ds, uint8_t *moved,
                                                       const uint32_t *fb_list, const uint32_t *fb_cnt) {
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
        moved[s] = bestv != old;
        if (ds) ds[s] = move_len(old, bestv, g);
      } else if (ds) {
        ds[s] = 0.0;
      }
    }
    __syncthreads();
  }
}
__global__ __launch_bounds__(256) void k_snap_fallback(const uint32_t *__restrict__ cell, Geom g, Sums sums,
                                                       uint32_t *sites, double *ds, uint8_t *moved,
                                                       const uint32_t *fb_list, const uint32_t *fb_cnt) { d_snap_fallback(cell, g, sums, sites, ds, moved, fb_list, fb_cnt); }


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

__device__ __forceinline__ void d_init_sites(const uint32_t *__restrict__ seeds, uint32_t S, const uint32_t *__restrict__ comp, Geom g,
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
__global__ void k_init_sites(const uint32_t *__restrict__ seeds, uint32_t S, const uint32_t *__restrict__ comp, Geom g,
                             uint32_t *sites, uint32_t *site_comp, uint32_t *err) { d_init_sites(seeds, S, comp, g, sites, site_comp, err); }


// ----------------------------------------------------------------------------
// host side

struct CvtWork {
  uint32_t *eq;
  uint16_t *fr, *vis, *yf;
  unsigned long long *xf;
  uint32_t *act, *ctl;  // brick marks; ctl[0..2] level alive flags, ctl[3] error bits, ctl[4] next wake level
  uint32_t *fb_list, *fb_cnt, *err;
  uint32_t *hist;
  uint32_t *cellb;           // [nbricks][4096] cells, brick-major (the search's own copy)
  uint32_t *dist;            // [nbricks][4096] hop distance of every reached voxel, brick-major
  uint16_t *inv;             // [nbricks][256] invalid voxels (incremental passes)
  uint32_t *bnd, *bcnt, *wake;  // kept-voxel lists per brick, their counts and wake levels
  uint8_t *moved;            // [S] site moved in the last update
  unsigned long long *xface; // [nbricks][2][256] packed x faces of the brick relaxation keys
  uint32_t *brlist;          // [nbricks] bricks of a relaxation round
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
  const bool inc = iters > 0;  // incremental passes follow the first one
  auto eq = a.template take<uint32_t>(nb * kRows * 3);
  auto fr = a.template take<uint16_t>(2 * nb * kRows);
  auto vis = a.template take<uint16_t>(nb * kRows);
  auto xf = a.template take<unsigned long long>(2 * nb * 8);
  auto yf = a.template take<uint16_t>(2 * nb * 32);
  auto act = a.template take<uint32_t>(2 * nb);
  auto ctl = a.template take<uint32_t>(8 + 2 * 8 + kHistLen);  // flags, diagnostic counters, visits per level
  auto fbl = a.template take<uint32_t>(s1);
  auto fbc = a.template take<uint32_t>(4);
  auto sums = a.template take<unsigned long long>(4 * s1);
  auto ds = a.template take<double>(s1);
  auto mean = a.template take<double>(iters > 0 ? iters : 1);
  auto mpart = a.template take<double>(kMeanParts);
  auto hist = a.template take<uint32_t>(kHistLen);
  auto cellb = a.template take<uint32_t>(nb * kRows * BX);
  auto dist = a.template take<uint32_t>(nb * kRows * BX);
  auto moved = a.template take<uint8_t>(s1);
  auto xface = a.template take<unsigned long long>(nb * 512);
  auto brlist = a.template take<uint32_t>(nb);
  auto inv = a.template take<uint16_t>(inc ? nb * kRows : 1);
  auto bnd = a.template take<uint32_t>(inc ? nb * kRows * BX : 1);
  auto bcnt = a.template take<uint32_t>(inc ? nb : 1);
  auto wake = a.template take<uint32_t>(inc ? nb : 1);
  if (W) {
    W->eq = eq;
    W->fr = fr;
    W->vis = vis;
    W->xf = xf;
    W->yf = yf;
    W->act = act;
    W->ctl = ctl;
    W->err = ctl + 3;
    W->fb_list = fbl;
    W->fb_cnt = fbc;
    W->sums = sums;
    W->ds = ds;
    W->mean = mean;
    W->mean_part = mpart;
    W->hist = hist;
    W->cellb = cellb;
    W->dist = dist;
    W->moved = moved;
    W->xface = xface;
    W->brlist = brlist;
    W->inv = inc ? inv : nullptr;
    W->bnd = inc ? bnd : nullptr;
    W->bcnt = inc ? bcnt : nullptr;
    W->wake = inc ? wake : nullptr;
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

// Captures kGraphRounds calls of launch_round(stream, position) into an executable
// graph (kernel nodes only: nothing is cleared by memset).  The capture runs
// on a stream of its own (the caller's may be the null stream, which cannot
// be captured); the graph is then launched on the caller's stream.
template <class F>
int32_t capture_rounds(hipGraphExec_t *exec, F launch_round) {
  hipStream_t cs = nullptr;
  LSRVT_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  int32_t rc = LSRVT_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    hipStreamDestroy(cs);
    return LSRVT_EDEVICE;
  }
  for (int i = 0; i < kGraphRounds && rc == LSRVT_OK; ++i) rc = launch_round(cs, i);
  const hipError_t e = hipStreamEndCapture(cs, &graph);
  hipStreamDestroy(cs);
  if (rc != LSRVT_OK || e != hipSuccess) {
    if (graph) hipGraphDestroy(graph);
    return rc ? rc : LSRVT_EDEVICE;
  }
  const hipError_t ei = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    *exec = nullptr;
    return LSRVT_EDEVICE;
  }
  return LSRVT_OK;
}

// Driver state of one Lloyd run: the levels or rounds of the previous
// passes, which size the first batch of launches of the next one, and the
// captured graphs of relaxation rounds.
struct VTState {
  uint32_t levels = 0;      // levels of the last full pass
  uint32_t inc_levels = 0;  // levels of the first run of the last incremental pass
  uint32_t br_rounds = 0;   // rounds of the last full brick relaxation pass
  uint32_t br_rounds_inc = 0;  // rounds of the last incremental one
  hipGraphExec_t br_graph = nullptr;  // kGraphRounds relaxation rounds of this call's workspace (narrow keys)
  hipGraphExec_t br_graph_w = nullptr;  // the same with wide keys
  bool keys_set = false;    // the key width of the brick relaxation is chosen at its first pass
  uint32_t id_bits = 0;     // narrow keys: the id field's bits; 0: wide keys
  VTState() = default;
  VTState(const VTState &) = delete;
  VTState &operator=(const VTState &) = delete;
  ~VTState() {
    if (br_graph) hipGraphExecDestroy(br_graph);
    if (br_graph_w) hipGraphExecDestroy(br_graph_w);
  }
};

// Which schedule computes the Voronoi passes: the level-synchronous search
// or the brick relaxation (both give the same regions bit for bit).  The
// choice is made per host thread (lsrvt_set_vt_engine); by default, the
// brick relaxation for volumes with many voxels per site (wide cells: many
// levels per pass, few relaxation rounds) and the level search otherwise.
enum class VTEngine { Auto = 0, Levels = 1, Bricks = 2 };

thread_local VTEngine t_engine = VTEngine::Auto;

VTEngine vt_engine(const Geom &g, uint32_t S) {
  VTEngine e = t_engine;
  if (e == VTEngine::Auto) {
    static const char *env = getenv("LSRVT_VT_ENGINE");
    if (env && env[0] == 'l') return VTEngine::Levels;
    if (env && env[0] == 'b') return VTEngine::Bricks;
    e = (S == 0 || g.n / (int64_t)S >= 1024) ? VTEngine::Bricks : VTEngine::Levels;
  }
  return e;
}

// Benchmark timing of the Voronoi passes' dominant kernel (levels or
// relaxation rounds): while enabled, an event pair on the launch stream
// around every batch of launches; read back by lsrvt_timing_read.
struct KernelTimer {
  std::mutex mu;
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending, pool;
  double ms = 0.0;
  uint64_t launches = 0;
  uint64_t passes = 0;
  int64_t voxels_per_pass = 0;
  int32_t engines = 0;  // bit 0: level passes recorded, bit 1: relaxation passes
};
// one timer per host thread: calls issued from different threads (streams)
// never share instrumentation state
KernelTimer &timer() {
  thread_local KernelTimer t;
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

// End of a pass: the brick-major cells are written to the caller's C-order
// cell array, row by row (16 contiguous voxels), with LSRVT_NONE for voxels
// never reached: in a full pass those of components without a site; in an
// incremental pass the invalid voxels not reached again (none: a moved site
// stays in its component), whose brick-major entry is set to NONE as well.
template <bool INC>
__global__ __launch_bounds__(kVTThreads) void k_vt_finish(const uint16_t *__restrict__ vis,
                                                          const uint16_t *__restrict__ inv, Geom g, VTGrid bg,
                                                          uint32_t *__restrict__ cellb, uint32_t *__restrict__ cell) {
  const int t = threadIdx.x;
  const int lx = t & 15;
  for (int64_t rr = (int64_t)blockIdx.x * (kVTThreads / BX) + (t >> 4); rr < bg.nbricks * kRows;
       rr += (int64_t)gridDim.x * (kVTThreads / BX)) {
    const int64_t b = rr / kRows;
    const int row = (int)(rr % kRows);
    const int bx = (int)(b % bg.nbx), by = (int)((b / bg.nbx) % bg.nby), bz = (int)(b / ((int64_t)bg.nbx * bg.nby));
    const int x = bx * BX + lx, y = by * BY + (row & 15), z = bz * BZ + (row >> 4);
    if (x >= g.nx || y >= g.ny || z >= g.nz) continue;
    const size_t bi = (size_t)rr * BX + lx;
    bool miss = !((vis[rr] >> lx) & 1u);
    if (INC) miss = miss && ((inv[rr] >> lx) & 1u);
    uint32_t c = cellb[bi];
    if (miss) {
      c = kNone;
      cellb[bi] = kNone;
    }
    cell[x + (int64_t)g.nx * (y + (int64_t)g.ny * z)] = c;
  }
}

// The same end of a level-search pass with the centroid sums of the update
// that follows, one workgroup per brick (segmented row scans, see Fuse).
template <bool INC>
__global__ __launch_bounds__(kVTThreads) void k_vt_finish_sums(const uint16_t *__restrict__ vis,
                                                               const uint16_t *__restrict__ inv, Geom g, VTGrid bg,
                                                               uint32_t *__restrict__ cellb,
                                                               uint32_t *__restrict__ cell, Fuse F) {
  __shared__ FinTab T;
  const int t = threadIdx.x;
  for (int64_t b = blockIdx.x; b < bg.nbricks; b += gridDim.x) {
    const int bx = (int)(b % bg.nbx), by = (int)((b / bg.nbx) % bg.nby), bz = (int)(b / ((int64_t)bg.nbx * bg.nby));
    fin_clear(T);
    __syncthreads();
#pragma unroll 4
    for (int i = 0; i < BX; ++i) {
      const int loc = i * kVTThreads + t;
      const int lx = loc & 15;
      const int64_t rr = b * kRows + (loc >> 4);
      const int x = bx * BX + lx, y = by * BY + ((loc >> 4) & 15), z = bz * BZ + (loc >> 8);
      const bool in = x < g.nx && y < g.ny && z < g.nz;
      const size_t bi = (size_t)b * (kRows * BX) + loc;
      uint32_t c = kNone;
      if (in) {
        bool miss = !((vis[rr] >> lx) & 1u);
        if (INC) miss = miss && ((inv[rr] >> lx) & 1u);
        c = cellb[bi];
        if (miss) {
          c = kNone;
          cellb[bi] = kNone;
        }
      }
      const int64_t v = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
      if (in) cell[v] = c;
      const uint32_t wv = in ? (F.w ? (uint32_t)F.w[v] : 1u) : 0u;
      fin_row_runs(T, F, c, wv, (uint32_t)(bx * BX), (uint32_t)y, (uint32_t)z);
    }
    __syncthreads();
    fin_flush(T, F);
  }
}

// Site voxels cleared before level 0 of a full pass (brick-major cells).
__global__ void k_sites_clear(const uint32_t *__restrict__ sites, uint32_t S, BFSArgs A) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S && (int64_t)sites[s] < A.g.n) A.cell[brick_pos(A, sites[s]).bi] = kNone;
}

unsigned brick_grid(const VTGrid &bg) { return (unsigned)std::min<int64_t>(bg.nbricks, 65535); }

// Workgroups of the relaxation's finish: one per slab of four x-adjacent bricks.
int64_t br_slabs(const VTGrid &bg) { return (int64_t)((bg.nbx + 3) / 4) * bg.nby * bg.nbz; }
unsigned slab_grid(const VTGrid &bg) { return (unsigned)std::min<int64_t>(br_slabs(bg), 65535); }

unsigned finish_grid(const VTGrid &bg) {
  const int64_t g = (bg.nbricks * kRows + kVTThreads / BX - 1) / (kVTThreads / BX);
  return (unsigned)(g < 65535 ? g : 65535);
}

int32_t vt_prepare(const uint8_t *band, const Geom &g, CvtWork &W, hipStream_t s) {
  VTGrid bg = vt_grid(g);
  const int64_t slots = bg.nbricks * kRows * BX;
  const unsigned grid = (unsigned)std::min<int64_t>((slots + kVTThreads - 1) / kVTThreads, 65535);
  hipLaunchKernelGGL(k_vt_eq, dim3(grid), dim3(kVTThreads), 0, s, band, g, bg, W.eq);
  LSRVT_LAUNCHED();
  return LSRVT_OK;
}

BFSArgs bfs_args(const Geom &g, CvtWork &W) {
  BFSArgs A;
  A.g = g;
  A.bg = vt_grid(g);
  A.eq = W.eq;
  A.fr = W.fr;
  A.vis = W.vis;
  A.xf = W.xf;
  A.yf = W.yf;
  A.cell = W.cellb;
  A.dist = W.dist;
  A.act = W.act;
  A.alive = W.ctl;
  A.hist = W.hist;
  A.err = W.err;
  A.inv = W.inv;
  A.bnd = W.bnd;
  A.bcnt = W.bcnt;
  A.wake = W.wake;
  static const bool debug_levels = getenv("LSRVT_DEBUG_LEVELS") != nullptr;
  A.dbg = debug_levels ? reinterpret_cast<unsigned long long *>(W.ctl + 8) : nullptr;
  return A;
}

// Clears the per-pass search state (frontiers, reached rows, marks, flags).
int32_t clear_pass(const VTGrid &bg, CvtWork &W, hipStream_t s) {
  int32_t rc;
  // 16-bit and 64-bit arrays are cleared as 32-bit words (even lengths)
  if ((rc = fill<uint32_t>(reinterpret_cast<uint32_t *>(W.fr), bg.nbricks * kRows, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(reinterpret_cast<uint32_t *>(W.vis), bg.nbricks * kRows / 2, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(reinterpret_cast<uint32_t *>(W.xf), 2 * bg.nbricks * 16, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(reinterpret_cast<uint32_t *>(W.yf), bg.nbricks * 32, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(W.act, 2 * bg.nbricks, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(W.ctl, 3, 0u, s))) return rc;
  return LSRVT_OK;
}

// Launches of the level kernel from level 1 on, enqueued in batches (the
// first one sized by the previous pass of the same kind, since sites move
// little between passes); after each batch the host reads the flags.  An
// incremental pass whose frontier dies out before every brick has injected
// its kept voxels continues at the smallest pending wake level.  Sets *redo
// when a kept-voxel list could not hold a level (the caller then runs a full
// pass).
template <bool INC>
int32_t run_levels(const Geom &g, const BFSArgs &A, CvtWork &W, VTState &st, hipStream_t s, bool *redo) {
  const VTGrid &bg = A.bg;
  const int64_t max_level = g.n + 2;
  const unsigned lgrid = (unsigned)std::min<int64_t>(8 * ((bg.nbricks + 7) / 8), 65528);
  const unsigned wgrid = (unsigned)std::min<int64_t>((bg.nbricks + 255) / 256, 1024);
  uint32_t L = 0;  // levels enqueued
  uint32_t run_end = 0;  // last level of the first run of consecutive launches
  bool jumped = false;
  int batch = INC ? (int)std::max<uint32_t>(8, st.inc_levels + 2) : (st.levels ? (int)st.levels + 4 : 16);
  int32_t rc;
  uint32_t c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  while (true) {
    // one event pair around a batch of back-to-back level launches (while
    // timing is on): the launches of a batch run without gaps
    const bool timed = timer().on;
    std::pair<hipEvent_t, hipEvent_t> ev;
    if (timed && (rc = timed_begin(s, ev))) return rc;
    for (int i = 0; i < batch; ++i) {
      ++L;
      hipLaunchKernelGGL(k_bfs_level<INC>, dim3(lgrid), dim3(kLvlThreads), 0, s, A, L);
      LSRVT_LAUNCHED();
    }
    if (timed && (rc = timed_end(s, ev, (uint64_t)batch))) return rc;
    if (INC) {
      if ((rc = fill<uint32_t>(W.ctl + 4, 1, kNone, s))) return rc;
      hipLaunchKernelGGL(k_wake_min, dim3(wgrid), dim3(256), 0, s, W.wake, bg.nbricks, W.ctl + 4);
      LSRVT_LAUNCHED();
    }
    if ((rc = read_words(W.ctl, 8, c, s))) return rc;
    const uint32_t e = c[3];
    if (INC && (e & 4u)) {
      *redo = true;
      return LSRVT_OK;
    }
    if (e & 1u) return LSRVT_EINVAL;
    if (e) return LSRVT_EDEVICE;
    if (!jumped) run_end = L;
    if (c[(L + 1) % 3] == 0) {  // no brick marked for the next level
      if (!INC || c[4] == kNone) break;
      // nothing marked until the next wake level: go there
      if ((rc = fill<uint32_t>(W.ctl, 3, 0u, s))) return rc;
      L = c[4] - 1;
      jumped = true;
    }
    if ((int64_t)L > max_level) return LSRVT_EDEVICE;
    batch = 8;
  }
  // the length of the first run of alive levels sizes the first batch of
  // the next pass of the same kind
  const uint32_t nl = std::min<uint32_t>(run_end + 1, kHistLen);
  std::vector<uint32_t> h(nl, 0);
  if (nl > 1) {
    LSRVT_HIP(hipMemcpyAsync(h.data(), W.hist, sizeof(uint32_t) * nl, hipMemcpyDeviceToHost, s));
    LSRVT_HIP(hipStreamSynchronize(s));
  }
  uint32_t levels = 0;
  while (levels + 1 < nl && h[levels + 1]) ++levels;
  (INC ? st.inc_levels : st.levels) = levels;
  static const bool debug_levels = getenv("LSRVT_DEBUG_LEVELS") != nullptr;
  if (debug_levels) {
    unsigned long long d[8];
    LSRVT_HIP(hipMemcpyAsync(d, W.ctl + 8, sizeof(d), hipMemcpyDeviceToHost, s));
    LSRVT_HIP(hipStreamSynchronize(s));
    fprintf(stderr, "[lsrvt] vt %s levels=%u last=%u visits=%llu cand=%llu big=%llu bigcand=%llu new=%llu inj=%llu\n",
            INC ? "inc" : "full", levels, L, d[0], d[1], d[2], d[3], d[4], d[5]);
    std::vector<uint32_t> pv(std::min<uint32_t>(L + 1, kHistLen));
    LSRVT_HIP(hipMemcpyAsync(pv.data(), W.ctl + 24, pv.size() * 4, hipMemcpyDeviceToHost, s));
    LSRVT_HIP(hipStreamSynchronize(s));
    fprintf(stderr, "[lsrvt]   visits per level:");
    for (size_t i = 1; i < pv.size(); ++i) fprintf(stderr, " %u", pv[i]);
    fprintf(stderr, "\n");
    if ((rc = fill<uint32_t>(W.ctl + 8, 2 * 8 + kHistLen, 0u, s))) return rc;
  }
  return LSRVT_OK;
}

// One restricted Voronoi pass over every voxel: level 0 at the sites, then
// the level launches until the device reports an empty level.
int32_t run_vt(const Geom &g, const uint32_t *sites, uint32_t S, uint32_t *cell, CvtWork &W, VTState &st,
               hipStream_t s, const Fuse *fz = nullptr) {
  VTGrid bg = vt_grid(g);
  int32_t rc;
  if ((rc = clear_pass(bg, W, s))) return rc;
  BFSArgs A = bfs_args(g, W);
  if (S) {
    hipLaunchKernelGGL(k_sites_clear, dim3((S + 255) / 256), dim3(256), 0, s, sites, S, A);
    hipLaunchKernelGGL(k_bfs_init, dim3((S + 255) / 256), dim3(256), 0, s, sites, S, A);
    LSRVT_LAUNCHED();
    bool redo = false;
    if ((rc = run_levels<false>(g, A, W, st, s, &redo))) return rc;
  }
  if (fz)
    hipLaunchKernelGGL(k_vt_finish_sums<false>, dim3(brick_grid(bg)), dim3(kVTThreads), 0, s, W.vis, W.inv, g, bg,
                       W.cellb, cell, *fz);
  else
    hipLaunchKernelGGL(k_vt_finish<false>, dim3(finish_grid(bg)), dim3(kVTThreads), 0, s, W.vis, W.inv, g, bg,
                       W.cellb, cell);
  LSRVT_LAUNCHED();
  if (timer().on) {
    std::lock_guard<std::mutex> lk(timer().mu);
    timer().passes += 1;
    timer().engines |= 1;
    timer().voxels_per_pass = g.n;
  }
  return LSRVT_OK;
}

// One incremental pass after an update: cell and dist hold the previous
// pass's keys and W.moved flags the sites that moved.  The result is that of
// a full pass with the new sites (see the incremental-pass notes above).
int32_t run_vt_inc(const Geom &g, const uint32_t *sites, uint32_t S, uint32_t *cell, CvtWork &W, VTState &st,
                   hipStream_t s, const Fuse *fz = nullptr) {
  if (!W.inv || S == 0) return run_vt(g, sites, S, cell, W, st, s, fz);
  VTGrid bg = vt_grid(g);
  int32_t rc;
  if ((rc = clear_pass(bg, W, s))) return rc;
  BFSArgs A = bfs_args(g, W);
  const int64_t slots = bg.nbricks * kRows * BX;
  const unsigned rgrid = (unsigned)std::min<int64_t>((slots + kVTThreads - 1) / kVTThreads, 65535);
  hipLaunchKernelGGL(k_inc_reset, dim3(rgrid), dim3(kVTThreads), 0, s, W.cellb, W.moved, g, bg, W.inv);
  hipLaunchKernelGGL(k_inc_site_a, dim3((S + 255) / 256), dim3(256), 0, s, sites, S, A);
  hipLaunchKernelGGL(k_inc_site_b, dim3((S + 255) / 256), dim3(256), 0, s, sites, S, A);
  hipLaunchKernelGGL(k_bnd_build, dim3((unsigned)std::min<int64_t>(bg.nbricks, 65535)), dim3(kLvlThreads), 0, s, A);
  LSRVT_LAUNCHED();
  bool redo = false;
  if ((rc = run_levels<true>(g, A, W, st, s, &redo))) return rc;
  if (redo) {
    if ((rc = fill<uint32_t>(W.err, 1, 0u, s))) return rc;
    return run_vt(g, sites, S, cell, W, st, s, fz);
  }
  if (fz)
    hipLaunchKernelGGL(k_vt_finish_sums<true>, dim3(brick_grid(bg)), dim3(kVTThreads), 0, s, W.vis, W.inv, g, bg,
                       W.cellb, cell, *fz);
  else
    hipLaunchKernelGGL(k_vt_finish<true>, dim3(finish_grid(bg)), dim3(kVTThreads), 0, s, W.vis, W.inv, g, bg,
                       W.cellb, cell);
  LSRVT_LAUNCHED();
  static const bool debug_levels = getenv("LSRVT_DEBUG_LEVELS") != nullptr;
  if (debug_levels) {  // sizes of the pass: moved sites, invalid and changed voxels, listed kept voxels
    std::vector<uint8_t> mv(S);
    std::vector<uint16_t> iv(bg.nbricks * kRows), vs(bg.nbricks * kRows);
    std::vector<uint32_t> bc(bg.nbricks);
    LSRVT_HIP(hipMemcpyAsync(mv.data(), W.moved, S, hipMemcpyDeviceToHost, s));
    LSRVT_HIP(hipMemcpyAsync(iv.data(), W.inv, iv.size() * 2, hipMemcpyDeviceToHost, s));
    LSRVT_HIP(hipMemcpyAsync(vs.data(), W.vis, vs.size() * 2, hipMemcpyDeviceToHost, s));
    LSRVT_HIP(hipMemcpyAsync(bc.data(), W.bcnt, bc.size() * 4, hipMemcpyDeviceToHost, s));
    LSRVT_HIP(hipStreamSynchronize(s));
    uint64_t nm = 0, ni = 0, nv = 0, nbd = 0, nbk = 0;
    for (uint8_t m : mv) nm += m != 0;
    for (size_t i = 0; i < iv.size(); ++i) {
      ni += __builtin_popcount(iv[i]);
      nv += __builtin_popcount(vs[i]);
    }
    for (uint32_t c : bc) {
      nbd += c;
      nbk += c != 0;
    }
    fprintf(stderr, "[lsrvt]   moved=%llu invalid=%llu changed=%llu kept-listed=%llu in %llu bricks\n",
            (unsigned long long)nm, (unsigned long long)ni, (unsigned long long)nv, (unsigned long long)nbd,
            (unsigned long long)nbk);
  }
  if (timer().on) {
    std::lock_guard<std::mutex> lk(timer().mu);
    timer().engines |= 1;
    timer().passes += 1;
    timer().voxels_per_pass = g.n;
  }
  return LSRVT_OK;
}

// The id bits of narrow relaxation keys for S sites, or 0 for wide keys.
// Narrow keys need the ids 0 .. S - 1 in b bits and, by default, keep at
// least 8 distance bits (b <= 24).  LSRVT_TUNE_KEY_BITS = 64 asks for wide
// keys; 1 .. 30 for narrow keys with an id field of at least that many bits.
uint32_t narrow_id_bits(uint32_t S) {
  const int32_t kb = tuning(LSRVT_TUNE_KEY_BITS);
  if (kb == 64) return 0;
  uint32_t b = 1;
  while (b < 32 && ((uint64_t)1 << b) < (uint64_t)S) ++b;
  if (kb > 0 && (uint32_t)kb > b) b = (uint32_t)kb;
  return b <= (kb > 0 ? 30u : 24u) ? b : 0u;
}

// Relaxation arguments over the workspace; id_bits: narrow keys with that
// id field, 0: wide keys.
BRArgs br_args(const Geom &g, CvtWork &W, uint32_t id_bits) {
  BRArgs A;
  A.moved = nullptr;
  A.fsites = nullptr;
  A.hop32 = id_bits ? 1u << id_bits : 0u;
  A.idmask = id_bits ? (1u << id_bits) - 1u : 0xFFFFFFFFu;
  A.lim32 = id_bits ? (uint32_t)(((uint64_t)1 << 32) - ((uint64_t)2 << id_bits)) : 0u;
  A.g = g;
  A.bg = vt_grid(g);
  A.eq = W.eq;
  A.key = W.cellb;  // spans the cell and distance arrays (room for wide keys)
  A.xface = W.xface;
  A.mark = W.act;
  A.list = W.brlist;
  A.rnd = W.ctl + 7;
  A.ctl = W.ctl;
  A.alive = W.ctl + 4;
  A.hist = W.hist;
  static const bool debug_levels = getenv("LSRVT_DEBUG_LEVELS") != nullptr;
  A.dbg = debug_levels ? reinterpret_cast<unsigned long long *>(W.ctl + 8) : nullptr;
  return A;
}

// One Voronoi pass by brick relaxation with keys KT: a full pass from the
// sites, or (inc) an incremental one from the previous keys after the
// update that set W.moved.  Rounds are enqueued in batches (the first sized
// by the previous pass); after each batch the host reads whether any brick
// is marked.  With narrow keys, a round that stored a key of the largest
// exact distance sets *far and the pass stops unfinished.
template <class KT>
int32_t run_br_k(const Geom &g, const uint32_t *sites, uint32_t S, uint32_t *cell, CvtWork &W, VTState &st,
                 bool inc, hipStream_t s, const Fuse *fz, bool *far) {
  const VTGrid bg = vt_grid(g);
  BRArgs A = br_args(g, W, sizeof(KT) == 4 ? st.id_bits : 0u);
  A.moved = W.moved;
  A.fsites = sites;
  constexpr KT kInf = BRKey<KT>::inf;
  int32_t rc;
  const int64_t nkeys = bg.nbricks * kRows * BX;
  if ((rc = fill<uint32_t>(W.act, 2 * bg.nbricks, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(W.ctl, 3, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(W.ctl + 4, 4, 0u, s))) return rc;  // alive flags and the round counter
  if (!inc) {
    if ((rc = fill<KT>(static_cast<KT *>(A.key), nkeys, kInf, s))) return rc;
    if ((rc = fill<KT>(static_cast<KT *>(A.xface), bg.nbricks * 512, kInf, s))) return rc;
  } else {
    hipLaunchKernelGGL(k_count_moved, dim3(std::min<uint32_t>((S + 255) / 256, 256) + (S == 0)), dim3(256), 0, s,
                       W.moved, S, W.ctl + 1);
    // The separate reset reads every key and lets round 1 work on the bricks
    // that hold reset voxels; the fused one costs about 1.5 rounds over
    // every brick.  A cube of the mean cell volume n / S overlaps about
    // (edge / 16 + 1)^3 bricks; the first round after a separate reset was
    // measured to work on far more (on the flame workload on nearly every
    // brick with 3 % of the sites moved: the reset bricks, the sites' bricks
    // and their neighbours), so eight times that count is taken, and the
    // fused reset once the moved sites would cover about 80 % of the bricks
    // by that estimate.
    const double edge = std::cbrt((double)g.n / std::max<uint32_t>(S, 1u));
    const double overlap = 8.0 * std::pow(edge / BX + 1.0, 3.0);
    const uint32_t fuse_min = (uint32_t)std::min(0.8 * (double)bg.nbricks / overlap, 4294967295.0);
    hipLaunchKernelGGL(k_br_reset_or_fuse<KT>, dim3((unsigned)std::min<int64_t>((nkeys + 255) / 256, 65535)),
                       dim3(256), 0, s, W.moved, A, fuse_min, tuning(LSRVT_TUNE_RESET));
    LSRVT_LAUNCHED();
  }
  if (S) {
    hipLaunchKernelGGL(k_br_sites<KT>, dim3((S + 255) / 256), dim3(256), 0, s, sites, S, A);
    LSRVT_LAUNCHED();
  }
  const unsigned lgrid = (unsigned)std::min<int64_t>((bg.nbricks + 255) / 256, 4096);
  const int32_t tg = tuning(LSRVT_TUNE_BR_GRID);
  const unsigned rgrid = (unsigned)std::min<int64_t>(bg.nbricks, tg ? tg : 2048);
  // kGraphRounds rounds (two launches each, and one that advances the
  // round base) captured once per call and replayed as one graph launch
  hipGraphExec_t &graph = sizeof(KT) == 4 ? st.br_graph : st.br_graph_w;
  if (!graph) {
    rc = capture_rounds(&graph, [&](hipStream_t cs, int i) -> int32_t {
      hipLaunchKernelGGL(k_br_list, dim3(lgrid), dim3(256), 0, cs, A, (int32_t)i);
      hipLaunchKernelGGL(k_br_round<KT>, dim3(rgrid), dim3(kBRThreads), 0, cs, A, (int32_t)i);
      if (i == kGraphRounds - 1) hipLaunchKernelGGL(k_br_advance, dim3(1), dim3(64), 0, cs, A);
      LSRVT_LAUNCHED();
      return LSRVT_OK;
    });
    if (rc) return rc;
  }
  uint32_t r = 0;
  uint32_t &hint = inc ? st.br_rounds_inc : st.br_rounds;
  int batch = hint ? (int)hint : inc ? 2 * kGraphRounds : kGraphRounds;
  uint32_t c[8];
  const int64_t max_rounds = 4 * g.n + 8;
  while (true) {
    const bool timed = timer().on;
    std::pair<hipEvent_t, hipEvent_t> ev;
    const int graphs = (batch + kGraphRounds - 1) / kGraphRounds;
    if (timed && (rc = timed_begin(s, ev))) return rc;
    for (int i = 0; i < graphs; ++i) LSRVT_HIP(hipGraphLaunch(graph, s));
    r += (uint32_t)(graphs * kGraphRounds);
    if (timed && (rc = timed_end(s, ev, (uint64_t)graphs * kGraphRounds))) return rc;
    if ((rc = read_words(W.ctl, 8, c, s))) return rc;
    if (c[3] & 1u) return LSRVT_EINVAL;
    if (c[3] & ~4u) return LSRVT_EDEVICE;
    if (c[3] & 4u) {  // a narrow key reached the largest exact distance
      *far = true;
      return LSRVT_OK;
    }
    if (c[4 + (r + 1) % 3] == 0) break;
    if ((int64_t)r > max_rounds) return LSRVT_EDEVICE;
    batch = kGraphRounds;
  }
  // the rounds that had work size the first batch of the next pass
  const uint32_t nl = std::min<uint32_t>(r + 1, kHistLen);
  std::vector<uint32_t> h(nl, 0);
  LSRVT_HIP(hipMemcpyAsync(h.data(), W.hist, sizeof(uint32_t) * nl, hipMemcpyDeviceToHost, s));
  LSRVT_HIP(hipStreamSynchronize(s));
  uint32_t worked = 0;
  while (worked + 1 < nl && h[worked + 1]) ++worked;
  hint = worked;
  static const bool debug_levels = getenv("LSRVT_DEBUG_LEVELS") != nullptr;
  if (debug_levels) {
    unsigned long long d[2];
    LSRVT_HIP(hipMemcpyAsync(d, W.ctl + 8, sizeof(d), hipMemcpyDeviceToHost, s));
    LSRVT_HIP(hipStreamSynchronize(s));
    if ((rc = fill<uint32_t>(W.ctl + 8, 4, 0u, s))) return rc;
    fprintf(stderr, "[lsrvt] br %s processings=%llu sweep rounds=%llu\n", inc ? "inc" : "full", d[0], d[1]);
    fprintf(stderr, "[lsrvt] br %s rounds=%u launched=%u bricks per round:", inc ? "inc" : "full", worked, r);
    for (uint32_t i = 1; i < nl; ++i) fprintf(stderr, " %u", h[i]);
    fprintf(stderr, "\n");
  }
  const KT *keys = static_cast<const KT *>(A.key);
  if (fz)
    hipLaunchKernelGGL(k_br_finish_sums<KT>, dim3(slab_grid(bg)), dim3(kVTThreads), 0, s, keys, g, bg, A.idmask,
                       cell, *fz);
  else
    hipLaunchKernelGGL(k_br_finish<KT>, dim3(slab_grid(bg)), dim3(kVTThreads), 0, s, keys, g, bg, A.idmask, cell);
  LSRVT_LAUNCHED();
  if (timer().on) {
    std::lock_guard<std::mutex> lk(timer().mu);
    timer().passes += 1;
    timer().voxels_per_pass = g.n;
    timer().engines |= 2;
  }
  return LSRVT_OK;
}

// One Voronoi pass by brick relaxation, with narrow keys when the sites
// allow and until a pass outgrows them: that pass is repeated from the sites
// with wide keys, which the rest of the call keeps.
int32_t run_br(const Geom &g, const uint32_t *sites, uint32_t S, uint32_t *cell, CvtWork &W, VTState &st, bool inc,
               hipStream_t s, const Fuse *fz = nullptr) {
  if (!st.keys_set) {
    st.id_bits = narrow_id_bits(S);
    st.keys_set = true;
  }
  if (st.id_bits) {
    bool far = false;
    int32_t rc = run_br_k<uint32_t>(g, sites, S, cell, W, st, inc, s, fz, &far);
    if (rc || !far) return rc;
    st.id_bits = 0;
    if ((rc = fill<uint32_t>(W.ctl + 3, 1, 0u, s))) return rc;
    inc = false;
  }
  return run_br_k<unsigned long long>(g, sites, S, cell, W, st, inc, s, fz, nullptr);
}

// A Voronoi pass with the selected schedule; with fz, its last kernel also
// takes the centroid sums of the update that follows.
int32_t vt_pass(const Geom &g, const uint32_t *sites, uint32_t S, uint32_t *cell, CvtWork &W, VTState &st, bool inc,
                hipStream_t s, const Fuse *fz = nullptr) {
  if (vt_engine(g, S) == VTEngine::Bricks) return run_br(g, sites, S, cell, W, st, inc, s, fz);
  return inc ? run_vt_inc(g, sites, S, cell, W, st, s, fz) : run_vt(g, sites, S, cell, W, st, s, fz);
}

// Errors a run reported on the device (synchronises).
int32_t vt_errors(CvtWork &W, hipStream_t s) {
  uint32_t e = 0;
  int32_t rc = read_words(W.err, 1, &e, s);
  if (rc) return rc;
  if (e & 1u) return LSRVT_EINVAL;
  if (e) return LSRVT_EDEVICE;
  return LSRVT_OK;
}

// The site update; with `summed` the centroid sums are already in W.sums
// (taken by the pass that produced the cells).
int32_t run_update(const uint32_t *cell, const Geom &g, const uint16_t *w, uint32_t *sites, uint32_t S, double *ds,
                   CvtWork &W, hipStream_t s, bool summed = false) {
  if (S == 0) return LSRVT_OK;
  int32_t rc;
  if ((rc = fill<uint32_t>(W.fb_cnt, 1, 0u, s))) return rc;
  Sums sm{W.sums, W.sums + S, W.sums + 2 * (size_t)S, W.sums + 3 * (size_t)S};
  if (!summed) {
    if ((rc = fill<unsigned long long>(W.sums, 4 * (int64_t)S, 0ull, s))) return rc;
    const int64_t ntiles = (int64_t)((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY) * ((g.nz + TZ - 1) / TZ);
    hipLaunchKernelGGL(k_centroid, dim3((unsigned)(ntiles < 65535 ? ntiles : 65535)), dim3(256), 0, s, cell, w, g, S,
                       sm);
  }
  hipLaunchKernelGGL(k_snap, dim3((S + 255) / 256), dim3(256), 0, s, cell, g, S, sm, sites, ds, W.moved, W.fb_list,
                     W.fb_cnt);
  hipLaunchKernelGGL(k_snap_fallback, dim3(S < 1024 ? S : 1024), dim3(256), 0, s, cell, g, sm, sites, ds, W.moved,
                     W.fb_list, W.fb_cnt);
  LSRVT_LAUNCHED();
  return LSRVT_OK;
}

int32_t begin(CvtWork &W, const Geom &g, hipStream_t s) {
  int32_t rc;
  VTGrid bg = vt_grid(g);
  if ((rc = fill<uint32_t>(W.act, 2 * bg.nbricks, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(W.ctl, 8 + 2 * 8 + kHistLen, 0u, s))) return rc;
  return LSRVT_OK;
}


// ----------------------------------------------------------------------------
// The Lloyd loops of many jobs in lockstep: every phase of every pass is one
// launch over all jobs (blockIdx.y = job), with each job's blocks striding
// over that job's own work.  The Voronoi passes use the brick relaxation
// (its rounds are shared: round r works on the marked bricks of every job,
// and the batch ends a pass when no job has a brick marked); a job with fewer
// updates than the batch's largest simply stops taking part.  Every job's
// kernels, sums and orders are its own, so its results are bit-identical to
// its lsrvt_cvt alone.
struct JobDev {
  BRArgs A;
  Geom g;
  const uint8_t *band;
  const uint32_t *comp, *seeds;
  const uint16_t *w;
  uint32_t *cell, *sites, *site_comp, *eq;
  uint32_t S;
  int32_t iters;
  Sums sums;
  double *ds;
  uint8_t *moved;
  uint32_t *fb_list, *fb_cnt;
};

__global__ __launch_bounds__(kVTThreads) void kb_vt_eq(const JobDev *J) {
  const JobDev &j = J[blockIdx.y];
  d_vt_eq(j.band, j.g, j.A.bg, j.eq);
}

__global__ void kb_init_sites(const JobDev *J) {
  const JobDev &j = J[blockIdx.y];
  d_init_sites(j.seeds, j.S, j.comp, j.g, j.sites, j.site_comp, j.A.ctl + 3);
}

// Start of pass t: marks and list counters cleared, and for a full pass
// (t = 0) every key and packed face unreached.  Block (0, 0) clears the
// shared round flags and round counter and records the pass (the shared
// words after the flags: [3] round, [4] pass, read by the graph-replayed
// round kernels).
template <class KT>
__global__ __launch_bounds__(256) void kb_pass_clear(const JobDev *J, int32_t t) {
  const JobDev &j = J[blockIdx.y];
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 5) j.A.alive[threadIdx.x] = threadIdx.x == 4 ? (uint32_t)t : 0u;
  if (t > j.iters) return;
  const int64_t nb = j.A.bg.nbricks, stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = i0; i < 2 * nb; i += stride) j.A.mark[i] = 0u;
  if (i0 == 0) j.A.ctl[0] = 0u;
  if (t == 0) {
    KT *key = static_cast<KT *>(j.A.key), *xface = static_cast<KT *>(j.A.xface);
    for (int64_t i = i0; i < nb * kRows * BX; i += stride) key[i] = BRKey<KT>::inf;
    for (int64_t i = i0; i < nb * 512; i += stride) xface[i] = BRKey<KT>::inf;
  }
}

template <class KT>
__global__ __launch_bounds__(256) void kb_reset(const JobDev *J, int32_t t) {
  const JobDev &j = J[blockIdx.y];
  if (t > j.iters || t == 0) return;
  d_br_reset<KT>(j.moved, j.A);
}

template <class KT>
__global__ void kb_sites(const JobDev *J, int32_t t) {
  const JobDev &j = J[blockIdx.y];
  if (t > j.iters) return;
  d_br_sites<KT>(j.sites, j.S, j.A);
}

// Start of a round: every job's list emptied, the shared round advanced.
__global__ void kb_round_prep(const JobDev *J) {
  if (threadIdx.x == 0) {
    const JobDev &j = J[blockIdx.y];
    j.A.ctl[0] = 0u;
    if (blockIdx.y == 0) j.A.alive[3] += 1u;
  }
}

__global__ __launch_bounds__(256) void kb_list(const JobDev *J) {
  const JobDev &j = J[blockIdx.y];
  if ((int32_t)j.A.alive[4] > j.iters) return;
  d_br_list(j.A, j.A.alive[3], &j.A.ctl[0]);
}

// The round's work list of the whole batch: the jobs' lists back to back,
// job j's at off[j] .. off[j + 1] (an exclusive prefix sum of the list
// counts, by one workgroup).  A job that has stopped taking part has an empty
// list.
__global__ __launch_bounds__(1024) void kb_offsets(const JobDev *J, int32_t n, uint32_t *off) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  const int32_t per = (n + 1023) / 1024, a = t * per, e = a + per < n ? a + per : n;
  const uint32_t r = J[0].A.alive[3];
  uint32_t sum = 0;
  for (int32_t i = a; i < e; ++i) {
    const uint32_t c = J[i].A.ctl[0];
    J[i].A.hist[r % kHistLen] = c;
    sum += c;
  }
  part[t] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive scan of the threads' sums
    const uint32_t v = t >= d ? part[t - d] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = part[t] - sum;
  for (int32_t i = a; i < e; ++i) {
    off[i] = run;
    run += J[i].A.ctl[0];
  }
  if (t == 1023) off[n] = part[1023];
}

// One relaxation round of the whole batch: the workgroups stride over the
// concatenated list, each item being a (job, brick) pair found by a binary
// search of the offsets.
template <class KT>
__global__ __launch_bounds__(kBRThreads, sizeof(KT) == 4 ? 5 : 4) void kb_round(const JobDev *J, int32_t n, const uint32_t *off) {
  __shared__ BRLds<KT> L;
  const uint32_t total = off[n];
  const uint32_t r = J[0].A.alive[3];
  for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
    int32_t lo = 0, hi = n - 1;  // the last job whose list starts at or before item
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (off[mid] <= item) lo = mid;
      else hi = mid - 1;
    }
    const BRArgs &A = J[lo].A;
    br_process<KT>(A, A.list[item - off[lo]], r, L);
  }
}

template <class KT>
__global__ __launch_bounds__(kVTThreads) void kb_finish(const JobDev *J, int32_t t) {
  const JobDev &j = J[blockIdx.y];
  if (t > j.iters) return;
  d_br_finish_slabs<KT, false>(static_cast<const KT *>(j.A.key), j.g, j.A.bg, j.A.idmask, j.cell, Fuse{}, nullptr);
}

__global__ __launch_bounds__(256) void kb_update_clear(const JobDev *J, int32_t t) {
  const JobDev &j = J[blockIdx.y];
  if (t >= j.iters) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = i0; i < 4 * (int64_t)j.S; i += stride) j.sums.M[i] = 0ull;  // M, Sx, Sy, Sz are contiguous
  if (i0 == 0) *j.fb_cnt = 0u;
}

__global__ __launch_bounds__(256) void kb_centroid(const JobDev *J, int32_t t) {
  const JobDev &j = J[blockIdx.y];
  if (t >= j.iters) return;
  d_centroid(j.cell, j.w, j.g, j.S, j.sums);
}

__global__ void kb_snap(const JobDev *J, int32_t t) {
  const JobDev &j = J[blockIdx.y];
  if (t >= j.iters) return;
  d_snap(j.cell, j.g, j.S, j.sums, j.sites, j.ds, j.moved, j.fb_list, j.fb_cnt);
}

__global__ __launch_bounds__(256) void kb_snap_fallback(const JobDev *J, int32_t t) {
  const JobDev &j = J[blockIdx.y];
  if (t >= j.iters) return;
  d_snap_fallback(j.cell, j.g, j.sums, j.sites, j.ds, j.moved, j.fb_list, j.fb_cnt);
}

}  // namespace

// Bytes of the descriptor block that precedes the jobs' workspaces.
// (the job descriptors, 256 bytes of shared round words, then the n + 1
// offsets of the batch's round list)
size_t cvt_batch_header(int32_t n) {
  return ((size_t)n * sizeof(JobDev) + 256 + 4 * ((size_t)n + 1) + 255) & ~size_t(255);
}

size_t cvt_batch_job_workspace(lsrvt_dims dims, uint32_t n_sites, int32_t iters) {
  Geom g;
  if (make_geom(dims, g)) return 0;
  return (cvt_workspace(g, n_sites, iters < 0 ? 0 : iters) + 255) & ~size_t(255);
}

namespace {

// What the lockstep loop needs besides the descriptors.
struct BatchCtx {
  int32_t n;
  JobDev *dj;           // device copy of the descriptors
  uint32_t *alive;      // shared round words
  uint32_t *offs;       // offsets of the batch's round list
  std::vector<JobDev> *hj;
  std::vector<CvtWork> *Ws;
  int32_t tmax;
  int64_t max_keys, max_sites, max_tiles, max_nb, max_slabs, sum_nb;
};

// The Lloyd loops of the batch with keys KT, from the seeds.  status[i]
// receives each job's status; *far is set when a job's narrow keys reached
// their largest exact distance (its results are then not to be used).
template <class KT>
int32_t batch_loop(const BatchCtx &c, int32_t *status, bool *far, hipStream_t s) {
  const int32_t n = c.n;
  JobDev *dj = c.dj;
  std::vector<JobDev> &hj = *c.hj;
  int32_t rc;
  LSRVT_HIP(hipMemcpyAsync(dj, hj.data(), sizeof(JobDev) * (size_t)n, hipMemcpyHostToDevice, s));
  for (int32_t i = 0; i < n; ++i)
    if ((rc = fill<uint32_t>((*c.Ws)[(size_t)i].ctl, 8 + 2 * 8, 0u, s))) return rc;
  const unsigned N = (unsigned)n;
  auto cap = [](int64_t v, int64_t m) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(v, m)); };
  const unsigned g_sites = cap((c.max_sites + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(kb_init_sites, dim3(g_sites, N), dim3(256), 0, s, dj);
  hipLaunchKernelGGL(kb_vt_eq, dim3(cap((c.max_keys + kVTThreads - 1) / kVTThreads, 65535), N), dim3(kVTThreads), 0,
                     s, dj);
  LSRVT_LAUNCHED();
  const unsigned g_clear = cap((c.max_keys + 255) / 256, 8192);
  const unsigned g_list = cap((c.max_nb + 255) / 256, 4096);
  const unsigned g_round = cap(c.sum_nb, tuning(LSRVT_TUNE_BR_GRID) > 0 ? tuning(LSRVT_TUNE_BR_GRID) : 2048);
  const unsigned g_fin = cap(c.max_slabs, 65535);
  const unsigned g_tiles = cap(c.max_tiles, 65535);
  const unsigned g_fb = cap(c.max_sites, 1024);
  uint32_t rounds_hint = 0;
  // kGraphRounds rounds of every job captured once and replayed as one graph launch
  VTState gs;
  uint32_t *offs = c.offs;
  rc = capture_rounds(&gs.br_graph, [&](hipStream_t cs, int) -> int32_t {
    hipLaunchKernelGGL(kb_round_prep, dim3(1, N), dim3(64), 0, cs, dj);
    hipLaunchKernelGGL(kb_list, dim3(g_list, N), dim3(256), 0, cs, dj);
    hipLaunchKernelGGL(kb_offsets, dim3(1), dim3(1024), 0, cs, dj, n, offs);
    hipLaunchKernelGGL(kb_round<KT>, dim3(g_round), dim3(kBRThreads), 0, cs, dj, n, (const uint32_t *)offs);
    LSRVT_LAUNCHED();
    return LSRVT_OK;
  });
  if (rc) return rc;
  for (int32_t t = 0; t <= c.tmax; ++t) {
    hipLaunchKernelGGL(kb_pass_clear<KT>, dim3(g_clear, N), dim3(256), 0, s, dj, t);
    if (t > 0) hipLaunchKernelGGL(kb_reset<KT>, dim3(g_clear, N), dim3(256), 0, s, dj, t);
    hipLaunchKernelGGL(kb_sites<KT>, dim3(g_sites, N), dim3(256), 0, s, dj, t);
    LSRVT_LAUNCHED();
    uint32_t r = 0;
    int batch = rounds_hint ? (int)rounds_hint : kGraphRounds;
    uint32_t w[3];
    const bool timed = timer().on;
    while (true) {
      std::pair<hipEvent_t, hipEvent_t> ev;
      const int graphs = (batch + kGraphRounds - 1) / kGraphRounds;
      if (timed && (rc = timed_begin(s, ev))) return rc;
      for (int k = 0; k < graphs; ++k) LSRVT_HIP(hipGraphLaunch(gs.br_graph, s));
      r += (uint32_t)(graphs * kGraphRounds);
      if (timed && (rc = timed_end(s, ev, (uint64_t)graphs * kGraphRounds))) return rc;
      if ((rc = read_words(c.alive, 3, w, s))) return rc;
      if (w[(r + 1) % 3] == 0) break;
      if (r > (uint32_t)(1u << 30)) return LSRVT_EDEVICE;
      batch = kGraphRounds;
    }
    rounds_hint = r;
    hipLaunchKernelGGL(kb_finish<KT>, dim3(g_fin, N), dim3(kVTThreads), 0, s, dj, t);
    if (t < c.tmax) {
      hipLaunchKernelGGL(kb_update_clear, dim3(g_sites, N), dim3(256), 0, s, dj, t);
      hipLaunchKernelGGL(kb_centroid, dim3(g_tiles, N), dim3(256), 0, s, dj, t);
      hipLaunchKernelGGL(kb_snap, dim3(g_sites, N), dim3(256), 0, s, dj, t);
      hipLaunchKernelGGL(kb_snap_fallback, dim3(g_fb, N), dim3(256), 0, s, dj, t);
    }
    LSRVT_LAUNCHED();
    if (timed) {
      std::lock_guard<std::mutex> lk(timer().mu);
      timer().engines |= 2;
      for (int32_t i = 0; i < n; ++i)
        if (t <= hj[(size_t)i].iters) {
          timer().passes += 1;
          timer().voxels_per_pass = hj[(size_t)i].g.n;
        }
    }
  }
  // each job's error bits (a seed outside its volume; a narrow key that
  // reached the largest exact distance)
  for (int32_t i = 0; i < n; ++i) {
    uint32_t e = 0;
    if ((rc = read_words((*c.Ws)[(size_t)i].ctl + 3, 1, &e, s))) return rc;
    if (e & 4u) *far = true;
    status[i] = (e & 1u) ? LSRVT_EINVAL : (e & ~4u) ? LSRVT_EDEVICE : LSRVT_OK;
  }
  return LSRVT_OK;
}

}  // namespace

// The Lloyd loops of n jobs in lockstep (see above).  work: the descriptor
// block, then one cvt workspace per job (cvt_batch_job_workspace each, in
// order).  status[i] receives each job's status.  Narrow relaxation keys
// are used when every job's sites allow them; if a job outgrows them, the
// batch is run again with wide keys.
int32_t cvt_batch(const CvtBatchJob *jobs, int32_t n, void *work, size_t bytes, int32_t *status, hipStream_t s) {
  if (n <= 0) return LSRVT_OK;
  std::vector<JobDev> hj((size_t)n);
  uint8_t *base = static_cast<uint8_t *>(work);
  const size_t head = cvt_batch_header(n);
  if (bytes < head) return LSRVT_EWORKSPACE;
  BatchCtx c{};
  c.n = n;
  c.dj = reinterpret_cast<JobDev *>(base);
  c.alive = reinterpret_cast<uint32_t *>(base + (size_t)n * sizeof(JobDev));
  c.offs = reinterpret_cast<uint32_t *>(base + (size_t)n * sizeof(JobDev) + 256);
  size_t off = head;
  std::vector<CvtWork> Ws((size_t)n);
  std::vector<uint32_t> bits((size_t)n);
  bool narrow = true;
  for (int32_t i = 0; i < n; ++i) {
    const CvtBatchJob &b = jobs[i];
    JobDev &j = hj[(size_t)i];
    Geom g;
    int32_t rc = make_geom(b.dims, g);
    if (rc) return rc;
    if (b.iters < 0 || !b.band || !b.comp || !b.cell || (b.n_sites && (!b.seeds || !b.sites || !b.site_comp)))
      return LSRVT_EINVAL;
    const size_t need = cvt_batch_job_workspace(b.dims, b.n_sites, b.iters);
    if (off + need > bytes) return LSRVT_EWORKSPACE;
    CvtWork &W = Ws[(size_t)i];
    if ((rc = carve_cvt(base + off, need, g, b.n_sites, b.iters, W))) return rc;
    off += need;
    bits[(size_t)i] = narrow_id_bits(b.n_sites);
    narrow = narrow && bits[(size_t)i] != 0;
    j.A = br_args(g, W, 0u);
    j.A.alive = c.alive;
    j.A.dbg = nullptr;
    j.g = g;
    j.band = b.band;
    j.comp = b.comp;
    j.seeds = b.seeds;
    j.w = b.weights;
    j.cell = b.cell;
    j.sites = b.sites;
    j.site_comp = b.site_comp;
    j.eq = W.eq;
    j.S = b.n_sites;
    j.iters = b.iters;
    const size_t S = b.n_sites;
    j.sums = Sums{W.sums, W.sums + S, W.sums + 2 * S, W.sums + 3 * S};
    j.ds = W.ds;
    j.moved = W.moved;
    j.fb_list = W.fb_list;
    j.fb_cnt = W.fb_cnt;
    c.tmax = std::max(c.tmax, b.iters);
    const VTGrid bg = vt_grid(g);
    c.max_nb = std::max<int64_t>(c.max_nb, bg.nbricks);
    c.sum_nb += bg.nbricks;
    c.max_keys = std::max<int64_t>(c.max_keys, bg.nbricks * kRows * BX);
    c.max_slabs = std::max<int64_t>(c.max_slabs, br_slabs(bg));
    c.max_sites = std::max<int64_t>(c.max_sites, (int64_t)S);
    c.max_tiles = std::max<int64_t>(c.max_tiles, (int64_t)((g.nx + TX - 1) / TX) * ((g.ny + TY - 1) / TY) *
                                                     ((g.nz + TZ - 1) / TZ));
  }
  c.hj = &hj;
  c.Ws = &Ws;
  if (narrow) {
    for (int32_t i = 0; i < n; ++i) {
      const BRArgs a = br_args(hj[(size_t)i].g, Ws[(size_t)i], bits[(size_t)i]);
      hj[(size_t)i].A.hop32 = a.hop32;
      hj[(size_t)i].A.idmask = a.idmask;
      hj[(size_t)i].A.lim32 = a.lim32;
    }
    bool far = false;
    const int32_t rc = batch_loop<uint32_t>(c, status, &far, s);
    if (rc || !far) return rc;
    for (int32_t i = 0; i < n; ++i) {
      const BRArgs a = br_args(hj[(size_t)i].g, Ws[(size_t)i], 0u);
      hj[(size_t)i].A.hop32 = a.hop32;
      hj[(size_t)i].A.idmask = a.idmask;
      hj[(size_t)i].A.lim32 = a.lim32;
    }
  }
  bool far = false;
  return batch_loop<unsigned long long>(c, status, &far, s);
}

namespace {
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
  if ((rc = vt_pass(g, d_sites, n_sites, d_cell, W, st, false, s))) return rc;
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
  const Fuse fz{d_weights, n_sites,
                Sums{W.sums, W.sums + n_sites, W.sums + 2 * (size_t)n_sites, W.sums + 3 * (size_t)n_sites}};
  for (int32_t t = 0; t <= iters; ++t) {
    // the first pass covers every voxel; later ones only what the moved sites change.  A pass
    // followed by an update also takes the update's centroid sums.
    const bool upd = t < iters && n_sites > 0;
    if (upd && (rc = fill<unsigned long long>(W.sums, 4 * (int64_t)n_sites, 0ull, s))) return rc;
    if ((rc = vt_pass(g, d_sites, n_sites, d_cell, W, st, t > 0, s, upd ? &fz : nullptr))) return rc;
    if (t == iters) break;
    if ((rc = run_update(d_cell, g, d_weights, d_sites, n_sites, W.ds, W, s, true))) return rc;
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

extern "C" int32_t lsrvt_timing_read(double *ms, uint64_t *launches, uint64_t *passes, int64_t *voxels_per_pass,
                                     int32_t *engines) {
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
  if (engines) *engines = T.engines;
  T.engines = 0;
  T.ms = 0.0;
  T.launches = 0;
  T.passes = 0;
  return LSRVT_OK;
}

// ----------------------------------------------------------------------------
// The site update for callers that cannot allocate device memory (code under
// graph capture, serving loops that forbid allocation): its scratch (per-site
// uint64 sums, the fallback list and counter, the moved flags) lives in a
// file-scope device array of fixed size, one copy per GPU, held until the
// process ends.  Host code never passes the array's name to a kernel: its
// device address is looked up once per device (with that device current)
// and kept.
namespace lsrvt {

constexpr uint32_t kNoAllocSites = LSRVT_UPDATE_NOALLOC_MAX_SITES;
constexpr size_t kNoAllocSums = (size_t)4 * kNoAllocSites * sizeof(unsigned long long);
constexpr size_t kNoAllocList = (size_t)kNoAllocSites * sizeof(uint32_t);
constexpr size_t kNoAllocBytes = kNoAllocSums + kNoAllocList + 256 + kNoAllocSites;

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

struct ScratchTable {
  std::mutex mu;
  std::vector<unsigned char *> ptr;  // device address of `scratch` per device (nullptr: not looked up)
};

ScratchTable &scratch_table() {
  static ScratchTable t;
  return t;
}

int32_t scratch_ptr(unsigned char **out) {
  int dev = 0;
  LSRVT_HIP(hipGetDevice(&dev));
  ScratchTable &T = scratch_table();
  std::lock_guard<std::mutex> lk(T.mu);
  if ((size_t)dev >= T.ptr.size()) T.ptr.resize((size_t)dev + 1, nullptr);
  if (!T.ptr[dev]) {
    void *p = nullptr;
    LSRVT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return LSRVT_EDEVICE;
    T.ptr[dev] = static_cast<unsigned char *>(p);
  }
  *out = T.ptr[dev];
  return LSRVT_OK;
}

}  // namespace
}  // namespace lsrvt

extern "C" int32_t lsrvt_update_noalloc(const uint32_t *d_cell, lsrvt_dims dims, const uint16_t *d_weights,
                                        uint32_t *d_sites, uint32_t n_sites, double *d_ds, void *stream) {
  Geom g;
  int32_t rc = make_geom(dims, g);
  if (rc) return rc;
  if (!d_cell || (n_sites && !d_sites)) return LSRVT_EINVAL;
  if (n_sites > kNoAllocSites) return LSRVT_ELIMIT;
  unsigned char *base = nullptr;
  if ((rc = scratch_ptr(&base))) return rc;
  CvtWork W{};
  W.sums = reinterpret_cast<unsigned long long *>(base);
  W.fb_list = reinterpret_cast<uint32_t *>(base + kNoAllocSums);
  W.fb_cnt = reinterpret_cast<uint32_t *>(base + kNoAllocSums + kNoAllocList);
  W.moved = base + kNoAllocSums + kNoAllocList + 256;
  return run_update(d_cell, g, d_weights, d_sites, n_sites, d_ds, W, as_stream(stream));
}

namespace lsrvt {
namespace {
thread_local int32_t t_tuning[5] = {0, 0, 0, 0, 0};
}  // namespace
int32_t tuning(int32_t knob) { return knob > 0 && knob < 5 ? t_tuning[knob] : 0; }
}  // namespace lsrvt

extern "C" int32_t lsrvt_set_tuning(int32_t knob, int32_t value) {
  if (knob == LSRVT_TUNE_BR_GRID) {
    if (value != 0 && (value < 256 || value > 16384)) return -1;
  } else if (knob == LSRVT_TUNE_STATS_TILE) {
    if (value != 0 && value != 1 && value != 2 && value != 4) return -1;
  } else if (knob == LSRVT_TUNE_KEY_BITS) {
    if (value != 64 && (value < 0 || value > 30)) return -1;
  } else if (knob == LSRVT_TUNE_RESET) {
    if (value < 0 || value > 2) return -1;
  } else {
    return -1;
  }
  const int32_t prev = t_tuning[knob];
  t_tuning[knob] = value;
  return prev;
}

extern "C" int32_t lsrvt_set_vt_engine(int32_t engine) {
  if (engine < 0 || engine > 2) return -1;
  const int32_t prev = (int32_t)t_engine;
  t_engine = (VTEngine)engine;
  return prev;
}
