// Restricted geodesic Voronoi pass (Eq. 1), snapped centroid update (Sec. 3.1
// "Centroids"; Sec. 3.2.3) and the fixed-iteration Lloyd loop (Algorithm 1).
//
// Voronoi pass.  Every voxel carries a 64-bit key (hop distance << 32 | site
// id).  The regions of Eq. 1 with ties to the lower id are the unique fixed
// point of key(v) = min(key(v), key(w) + (1 << 32)) over same-band face
// neighbours w, started from key = (0, s) at every site and +inf elsewhere:
// every key is the length of a real path, so it never undercuts the true
// lexicographic minimum, and at a fixed point the minimum is reached along
// any shortest path.  Because the fixed point is unique, relaxations may run
// in any order and the result is bit-deterministic.
//
// The volume is cut into 16^3 bricks.  A round relaxes a list of bricks, one
// workgroup each: the brick's bands and keys sit in LDS, its own sites and
// the keys its six neighbours last published on their facing faces seed it,
// and alternating forward/backward line sweeps along x, y and z (each a
// min-plus scan over a same-band run) repeat until nothing changes.  The
// brick then writes its cells and publishes its six faces; a neighbour is
// queued for the next round only if a facing face key changed.  The first
// round of a pass processes every brick without halos.  Rounds repeat until
// no brick is queued.
//
// Update.  Per site, M = sum w and S_a = sum w a are exact uint64 sums
// (wave-aggregated atomics).  The nearest lattice point to S/M with ties
// rounded down, q_a = floor((2 S_a + M - 1) / (2 M)), is the answer whenever
// it lies in the cell (it then minimises the distance over all lattice
// points, and among tied points the all-lower corner has the smallest linear
// index).  Otherwise one workgroup searches cubes of growing half-width r
// around q; voxels outside the cube are at least r + 1/2 from the centroid,
// so the search stops once 4 D_best < (M (2 r + 1))^2, comparing
// D = sum_a (M a - S_a)^2 exactly in 128 bits.
#include "common.h"

namespace lsrvt {

namespace {

constexpr int BX = 16, BY = 16, BZ = 16;
constexpr int PX = BX + 1;  // padded LDS pitch (u64 elements) for conflict-free x sweeps
constexpr int kBrickVox = BX * BY * BZ;
constexpr int kVTThreads = 256;
constexpr int kFaceLen = 256;  // every face of a 16^3 brick has 256 voxels
constexpr int kFaces = 6;
constexpr uint64_t kD1 = 1ull << 32;
constexpr uint8_t kOutside = 255;
constexpr int kMaxSweepCycles = 1 << 14;

struct VTGrid {
  int32_t nbx, nby, nbz;
  int64_t nbricks;
};

struct VTArgs {
  const uint8_t *band;
  Geom g;
  VTGrid bg;
  const uint32_t *sites;
  const uint32_t *blist;  // site ids bucketed by brick
  const uint32_t *boff;   // [nbricks + 1]
  const uint8_t *site_band;
  uint64_t *faces;        // [nbricks][6][256]
  uint32_t *cell;
  uint32_t *queued;       // [nbricks] last epoch tag
  uint32_t *list_in;
  uint32_t *list_out;
  uint32_t *cnt;          // [3] rotating list counters
  uint32_t *err;
};

__device__ __forceinline__ int kidx(int lx, int ly, int lz) { return (lz * BY + ly) * PX + lx; }
__device__ __forceinline__ int bidx(int lx, int ly, int lz) { return (lz * BY + ly) * BX + lx; }

// Face f of a brick: 0:-x 1:+x (index [lz][ly]), 2:-y 3:+y ([lz][lx]), 4:-z 5:+z ([ly][lx]).
__device__ __forceinline__ void face_voxel(int f, int p, int &lx, int &ly, int &lz) {
  int a = p & 15, c = p >> 4;
  switch (f) {
    case 0: lx = 0; ly = a; lz = c; break;
    case 1: lx = BX - 1; ly = a; lz = c; break;
    case 2: lx = a; ly = 0; lz = c; break;
    case 3: lx = a; ly = BY - 1; lz = c; break;
    case 4: lx = a; ly = c; lz = 0; break;
    default: lx = a; ly = c; lz = BZ - 1; break;
  }
}

__global__ __launch_bounds__(kVTThreads) void k_vt_round(VTArgs A, uint32_t epoch, int all) {
  __shared__ uint64_t key[BZ * BY * PX];
  __shared__ uint8_t bnd[kBrickVox];
  __shared__ int s_changed;
  __shared__ uint32_t s_count;
  const int t = threadIdx.x;
  if (t == 0) {
    s_count = all ? (uint32_t)A.bg.nbricks : A.cnt[epoch % 3];
    if (blockIdx.x == 0) A.cnt[(epoch + 2) % 3] = 0;  // the list the round after next appends to
  }
  __syncthreads();
  const uint32_t count = s_count;
  uint32_t *out_cnt = &A.cnt[(epoch + 1) % 3];

  for (uint32_t item = blockIdx.x; item < count; item += gridDim.x) {
    const uint32_t b = all ? item : A.list_in[item];
    const int bx = (int)(b % A.bg.nbx), by = (int)((b / A.bg.nbx) % A.bg.nby), bz = (int)(b / ((uint32_t)A.bg.nbx * A.bg.nby));
    const int x0 = bx * BX, y0 = by * BY, z0 = bz * BZ;
    // bands and +inf keys
    for (int li = t; li < kBrickVox; li += kVTThreads) {
      int lx = li & 15, ly = (li >> 4) & 15, lz = li >> 8;
      int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
      bool valid = gx < A.g.nx && gy < A.g.ny && gz < A.g.nz;
      bnd[li] = valid ? A.band[gx + (int64_t)A.g.nx * (gy + (int64_t)A.g.ny * gz)] : kOutside;
      key[kidx(lx, ly, lz)] = kInfKey;
    }
    __syncthreads();
    // own sites at distance 0 (co-located sites: the lower id wins the min)
    for (uint32_t i = A.boff[b] + t; i < A.boff[b + 1]; i += kVTThreads) {
      uint32_t s = A.blist[i];
      uint32_t v = A.sites[s];
      int gx = (int)(v % (uint32_t)A.g.nx);
      uint32_t r = v / (uint32_t)A.g.nx;
      int gy = (int)(r % (uint32_t)A.g.ny), gz = (int)(r / (uint32_t)A.g.ny);
      atomicMin((unsigned long long *)&key[kidx(gx - x0, gy - y0, gz - z0)], (unsigned long long)s);
    }
    // halo: the keys the neighbours published on the faces facing this brick
    if (!all) {
      for (int f = 0; f < kFaces; ++f) {
        int nbx = bx + (f == 0 ? -1 : f == 1 ? 1 : 0);
        int nby = by + (f == 2 ? -1 : f == 3 ? 1 : 0);
        int nbz = bz + (f == 4 ? -1 : f == 5 ? 1 : 0);
        if (nbx < 0 || nby < 0 || nbz < 0 || nbx >= A.bg.nbx || nby >= A.bg.nby || nbz >= A.bg.nbz) continue;
        int64_t nb = nbx + (int64_t)A.bg.nbx * (nby + (int64_t)A.bg.nby * nbz);
        const uint64_t *src = A.faces + (nb * kFaces + (f ^ 1)) * kFaceLen;
        uint64_t kv = src[t];
        if (kv != kInfKey) {
          int lx, ly, lz;
          face_voxel(f, t, lx, ly, lz);
          uint8_t mb = bnd[bidx(lx, ly, lz)];
          if (mb != kOutside && A.site_band[(uint32_t)kv] == mb)
            atomicMin((unsigned long long *)&key[kidx(lx, ly, lz)], (unsigned long long)(kv + kD1));
        }
      }
    }
    __syncthreads();

    // relax: x, y, z line sweeps until a full cycle changes nothing
    int cycles = 0;
    while (true) {
      bool ch = false;
      {  // x lines
        const int ly = t & 15, lz = t >> 4;
        uint64_t *row = &key[kidx(0, ly, lz)];
        const uint8_t *br = &bnd[bidx(0, ly, lz)];
        uint64_t k[BX];
        uint8_t bb[BX];
#pragma unroll
        for (int x = 0; x < BX; ++x) {
          k[x] = row[x];
          bb[x] = br[x];
        }
        bool c = false;
#pragma unroll
        for (int x = 1; x < BX; ++x)
          if (bb[x] == bb[x - 1] && k[x - 1] + kD1 < k[x] && k[x - 1] != kInfKey) {
            k[x] = k[x - 1] + kD1;
            c = true;
          }
#pragma unroll
        for (int x = BX - 2; x >= 0; --x)
          if (bb[x] == bb[x + 1] && k[x + 1] + kD1 < k[x] && k[x + 1] != kInfKey) {
            k[x] = k[x + 1] + kD1;
            c = true;
          }
        if (c) {
#pragma unroll
          for (int x = 0; x < BX; ++x) row[x] = k[x];
        }
        ch |= c;
      }
      __syncthreads();
      {  // y lines
        const int lx = t & 15, lz = t >> 4;
        uint64_t k[BY];
        uint8_t bb[BY];
#pragma unroll
        for (int y = 0; y < BY; ++y) {
          k[y] = key[kidx(lx, y, lz)];
          bb[y] = bnd[bidx(lx, y, lz)];
        }
        bool c = false;
#pragma unroll
        for (int y = 1; y < BY; ++y)
          if (bb[y] == bb[y - 1] && k[y - 1] + kD1 < k[y] && k[y - 1] != kInfKey) {
            k[y] = k[y - 1] + kD1;
            c = true;
          }
#pragma unroll
        for (int y = BY - 2; y >= 0; --y)
          if (bb[y] == bb[y + 1] && k[y + 1] + kD1 < k[y] && k[y + 1] != kInfKey) {
            k[y] = k[y + 1] + kD1;
            c = true;
          }
        if (c) {
#pragma unroll
          for (int y = 0; y < BY; ++y) key[kidx(lx, y, lz)] = k[y];
        }
        ch |= c;
      }
      __syncthreads();
      {  // z lines
        const int lx = t & 15, ly = t >> 4;
        uint64_t k[BZ];
        uint8_t bb[BZ];
#pragma unroll
        for (int z = 0; z < BZ; ++z) {
          k[z] = key[kidx(lx, ly, z)];
          bb[z] = bnd[bidx(lx, ly, z)];
        }
        bool c = false;
#pragma unroll
        for (int z = 1; z < BZ; ++z)
          if (bb[z] == bb[z - 1] && k[z - 1] + kD1 < k[z] && k[z - 1] != kInfKey) {
            k[z] = k[z - 1] + kD1;
            c = true;
          }
#pragma unroll
        for (int z = BZ - 2; z >= 0; --z)
          if (bb[z] == bb[z + 1] && k[z + 1] + kD1 < k[z] && k[z + 1] != kInfKey) {
            k[z] = k[z + 1] + kD1;
            c = true;
          }
        if (c) {
#pragma unroll
          for (int z = 0; z < BZ; ++z) key[kidx(lx, ly, z)] = k[z];
        }
        ch |= c;
      }
      int any = __syncthreads_or(ch ? 1 : 0);
      if (!any) break;
      if (++cycles >= kMaxSweepCycles) {
        if (t == 0) atomicOr(A.err, 2u);
        break;
      }
    }

    // cells
    for (int li = t; li < kBrickVox; li += kVTThreads) {
      int lx = li & 15, ly = (li >> 4) & 15, lz = li >> 8;
      int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
      if (gx < A.g.nx && gy < A.g.ny && gz < A.g.nz) {
        uint64_t kv = key[kidx(lx, ly, lz)];
        A.cell[gx + (int64_t)A.g.nx * (gy + (int64_t)A.g.ny * gz)] = kv == kInfKey ? kNone : (uint32_t)kv;
      }
    }
    // publish faces; queue a neighbour when a facing key changed
    for (int f = 0; f < kFaces; ++f) {
      int nbx = bx + (f == 0 ? -1 : f == 1 ? 1 : 0);
      int nby = by + (f == 2 ? -1 : f == 3 ? 1 : 0);
      int nbz = bz + (f == 4 ? -1 : f == 5 ? 1 : 0);
      bool exists = !(nbx < 0 || nby < 0 || nbz < 0 || nbx >= A.bg.nbx || nby >= A.bg.nby || nbz >= A.bg.nbz);
      if (!exists) continue;  // uniform across the workgroup
      int lx, ly, lz;
      face_voxel(f, t, lx, ly, lz);
      uint64_t kv = key[kidx(lx, ly, lz)];
      uint64_t *dst = A.faces + ((int64_t)b * kFaces + f) * kFaceLen;
      bool diff;
      if (all) {
        diff = kv != kInfKey;
        dst[t] = kv;
      } else {
        uint64_t old = dst[t];
        diff = kv != old;
        if (diff) dst[t] = kv;
      }
      int any = __syncthreads_or(diff ? 1 : 0);
      if (any && t == 0) {
        uint32_t nb = (uint32_t)(nbx + A.bg.nbx * (nby + A.bg.nby * nbz));
        uint32_t old = atomicMax(&A.queued[nb], epoch + 1);
        if (old < epoch + 1) {
          uint32_t pos = atomicAdd(out_cnt, 1u);
          A.list_out[pos] = nb;
        }
      }
    }
    __syncthreads();
  }
}

// Sites: count per brick and note each site's band; out-of-range sites are
// reported through err and left out.
__global__ void k_site_count(const uint32_t *__restrict__ sites, uint32_t S, const uint8_t *__restrict__ band, Geom g,
                             VTGrid bg, uint32_t *bcount, uint8_t *site_band, uint32_t *err) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  uint32_t v = sites[s];
  if ((int64_t)v >= g.n) {
    atomicOr(err, 1u);
    site_band[s] = kOutside;
    return;
  }
  uint32_t x = v % (uint32_t)g.nx, r = v / (uint32_t)g.nx;
  uint32_t y = r % (uint32_t)g.ny, z = r / (uint32_t)g.ny;
  uint32_t b = x / BX + bg.nbx * (y / BY + bg.nby * (z / BZ));
  atomicAdd(&bcount[b], 1u);
  site_band[s] = band[v];
}

__global__ void k_site_fill(const uint32_t *__restrict__ sites, uint32_t S, Geom g, VTGrid bg,
                            const uint32_t *__restrict__ boff, uint32_t *bfill, uint32_t *blist) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  uint32_t v = sites[s];
  if ((int64_t)v >= g.n) return;
  uint32_t x = v % (uint32_t)g.nx, r = v / (uint32_t)g.nx;
  uint32_t y = r % (uint32_t)g.ny, z = r / (uint32_t)g.ny;
  uint32_t b = x / BX + bg.nbx * (y / BY + bg.nby * (z / BZ));
  uint32_t pos = boff[b] + atomicAdd(&bfill[b], 1u);
  blist[pos] = s;
}

// ----------------------------------------------------------------------------
// update

struct Sums {
  unsigned long long *M, *Sx, *Sy, *Sz;
};

// One wave per row (y, z) at a time; along the row the wave takes 64 voxels per
// step, and equal cell ids inside the step are reduced before the atomics.
// Along a row y and z are fixed, so S_y = M y and S_z = M z.
__global__ __launch_bounds__(kWave) void k_centroid(const uint32_t *__restrict__ cell, const uint16_t *__restrict__ w,
                                                    Geom g, uint32_t S, Sums sums) {
  const int64_t rows = (int64_t)g.ny * g.nz;
  const int lane = lane_id();
  for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const uint64_t y = (uint64_t)(row % g.ny), z = (uint64_t)(row / g.ny);
    const int64_t base = row * g.nx;
    for (int x0 = 0; x0 < g.nx; x0 += kWave) {
      int x = x0 + lane;
      bool valid = x < g.nx;
      uint32_t c = valid ? cell[base + x] : kNone;
      uint64_t wv = 0;
      if (valid && c != kNone && c < S) wv = w ? (uint64_t)w[base + x] : 1ull;
      bool pending = valid && c != kNone && c < S;
      while (true) {
        uint64_t act = __ballot(pending);
        if (!act) break;
        int leader = __ffsll((long long)act) - 1;
        uint32_t c0 = __shfl(c, leader, kWave);
        bool mine = pending && c == c0;
        uint64_t m = wave_sum_u64(mine ? wv : 0ull);
        uint64_t sx = wave_sum_u64(mine ? wv * (uint64_t)x : 0ull);
        if (lane == leader && m) {
          atomicAdd(&sums.M[c0], (unsigned long long)m);
          atomicAdd(&sums.Sx[c0], (unsigned long long)sx);
          atomicAdd(&sums.Sy[c0], (unsigned long long)(m * y));
          atomicAdd(&sums.Sz[c0], (unsigned long long)(m * z));
        }
        pending = pending && !mine;
      }
    }
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

// Mean of ds[0..S) in a fixed order (one workgroup).
__global__ __launch_bounds__(256) void k_mean_ds(const double *ds, uint32_t S, double *out) {
  __shared__ double part[256];
  double acc = 0.0;
  for (uint32_t i = threadIdx.x; i < S; i += 256) acc += ds[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = S ? part[0] / (double)S : 0.0;
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
  uint64_t *faces;
  uint32_t *queued, *list_a, *list_b, *cnt, *bcount, *boff, *bfill, *blist, *fb_list, *fb_cnt, *err;
  uint8_t *site_band;
  unsigned long long *sums;  // 4 x S
  double *ds, *mean;
  void *scan_work;
  size_t scan_bytes;
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
  auto faces = a.template take<uint64_t>(nb * kFaces * kFaceLen);
  auto queued = a.template take<uint32_t>(nb);
  auto la = a.template take<uint32_t>(nb);
  auto lb = a.template take<uint32_t>(nb);
  auto cnt = a.template take<uint32_t>(4);
  auto bcount = a.template take<uint32_t>(nb);
  auto boff = a.template take<uint32_t>(nb + 1);
  auto bfill = a.template take<uint32_t>(nb);
  auto blist = a.template take<uint32_t>(s1);
  auto fbl = a.template take<uint32_t>(s1);
  auto fbc = a.template take<uint32_t>(4);
  auto err = a.template take<uint32_t>(4);
  auto sb = a.template take<uint8_t>(s1);
  auto sums = a.template take<unsigned long long>(4 * s1);
  auto ds = a.template take<double>(s1);
  auto mean = a.template take<double>(iters > 0 ? iters : 1);
  if (W) {
    W->faces = faces;
    W->queued = queued;
    W->list_a = la;
    W->list_b = lb;
    W->cnt = cnt;
    W->bcount = bcount;
    W->boff = boff;
    W->bfill = bfill;
    W->blist = blist;
    W->fb_list = fbl;
    W->fb_cnt = fbc;
    W->err = err;
    W->site_band = sb;
    W->sums = sums;
    W->ds = ds;
    W->mean = mean;
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
  return z.off + ScanU32::workspace(vt_grid(g).nbricks + 1) + 256;
}

int32_t carve_cvt(void *d_work, size_t bytes, const Geom &g, uint32_t S, int32_t iters, CvtWork &W) {
  Carve cv(d_work, bytes);
  cvt_layout(cv, g, S, iters, &W);
  if (!cv.ok) return LSRVT_EWORKSPACE;
  W.scan_work = cv.base + cv.off;
  W.scan_bytes = cv.size - cv.off;
  return LSRVT_OK;
}

// Driver state of one Lloyd run (epochs and a round-count hint).
struct VTState {
  uint32_t epoch = 1;
  int rounds_hint = 4;
};

int32_t read_u32(const uint32_t *d, uint32_t &h, hipStream_t s) {
  LSRVT_HIP(hipMemcpyAsync(&h, d, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  LSRVT_HIP(hipStreamSynchronize(s));
  return LSRVT_OK;
}

int32_t run_vt(const uint8_t *band, const Geom &g, const uint32_t *sites, uint32_t S, uint32_t *cell, CvtWork &W,
               VTState &st, hipStream_t s) {
  VTGrid bg = vt_grid(g);
  int32_t rc;
  // bucket the sites by brick
  if ((rc = fill<uint32_t>(W.bcount, bg.nbricks, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(W.bfill, bg.nbricks, 0u, s))) return rc;
  if (S) {
    hipLaunchKernelGGL(k_site_count, dim3((S + 255) / 256), dim3(256), 0, s, sites, S, band, g, bg, W.bcount,
                       W.site_band, W.err);
    LSRVT_LAUNCHED();
  }
  if ((rc = ScanU32::run(W.bcount, bg.nbricks, W.boff, W.scan_work, W.scan_bytes, s))) return rc;
  if (S) {
    hipLaunchKernelGGL(k_site_fill, dim3((S + 255) / 256), dim3(256), 0, s, sites, S, g, bg, W.boff, W.bfill, W.blist);
    LSRVT_LAUNCHED();
  }
  VTArgs A;
  A.band = band;
  A.g = g;
  A.bg = bg;
  A.sites = sites;
  A.blist = W.blist;
  A.boff = W.boff;
  A.site_band = W.site_band;
  A.faces = W.faces;
  A.cell = cell;
  A.queued = W.queued;
  A.cnt = W.cnt;
  A.err = W.err;
  const unsigned grid_all = (unsigned)(bg.nbricks < 65535 ? bg.nbricks : 65535);
  const unsigned grid_list = (unsigned)(bg.nbricks < 2048 ? bg.nbricks : 2048);
  const int64_t max_rounds = 2 * bg.nbricks + 16;
  int64_t done_rounds = 0;
  bool first = true;
  int batch = st.rounds_hint;
  while (true) {
    for (int i = 0; i < batch; ++i) {
      bool all = first;
      A.list_in = (st.epoch & 1) ? W.list_a : W.list_b;
      A.list_out = (st.epoch & 1) ? W.list_b : W.list_a;
      hipLaunchKernelGGL(k_vt_round, dim3(all ? grid_all : grid_list), dim3(kVTThreads), 0, s, A, st.epoch,
                         all ? 1 : 0);
      LSRVT_LAUNCHED();
      ++st.epoch;
      ++done_rounds;
      first = false;
    }
    uint32_t pending = 0, err = 0;
    if ((rc = read_u32(&W.cnt[st.epoch % 3], pending, s))) return rc;
    if ((rc = read_u32(W.err, err, s))) return rc;
    if (err & 1u) return LSRVT_EINVAL;
    if (err) return LSRVT_EDEVICE;
    if (pending == 0) break;
    if (done_rounds > max_rounds) return LSRVT_EDEVICE;
    batch = 2;
  }
  st.rounds_hint = (int)(done_rounds < 2 ? 2 : done_rounds);
  return LSRVT_OK;
}

int32_t run_update(const uint32_t *cell, const Geom &g, const uint16_t *w, uint32_t *sites, uint32_t S, double *ds,
                   CvtWork &W, hipStream_t s) {
  if (S == 0) return LSRVT_OK;
  int32_t rc;
  if ((rc = fill<unsigned long long>(W.sums, 4 * (int64_t)S, 0ull, s))) return rc;
  if ((rc = fill<uint32_t>(W.fb_cnt, 1, 0u, s))) return rc;
  Sums sm{W.sums, W.sums + S, W.sums + 2 * (size_t)S, W.sums + 3 * (size_t)S};
  int64_t rows = (int64_t)g.ny * g.nz;
  hipLaunchKernelGGL(k_centroid, dim3((unsigned)(rows < 262144 ? rows : 262144)), dim3(kWave), 0, s, cell, w, g, S, sm);
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
  if ((rc = fill<uint32_t>(W.cnt, 4, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(W.err, 1, 0u, s))) return rc;
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
  VTState st;
  return run_vt(d_band, g, d_sites, n_sites, d_cell, W, st, s);
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
  VTState st;
  for (int32_t t = 0; t <= iters; ++t) {
    if ((rc = run_vt(d_band, g, d_sites, n_sites, d_cell, W, st, s))) return rc;
    if (t == iters) break;
    if ((rc = run_update(d_cell, g, d_weights, d_sites, n_sites, W.ds, W, s))) return rc;
    hipLaunchKernelGGL(k_mean_ds, dim3(1), dim3(256), 0, s, W.ds, n_sites, W.mean + t);
    LSRVT_LAUNCHED();
  }
  if (h_mean_ds && iters > 0) {
    LSRVT_HIP(hipMemcpyAsync(h_mean_ds, W.mean, sizeof(double) * iters, hipMemcpyDeviceToHost, s));
    LSRVT_HIP(hipStreamSynchronize(s));
  }
  return LSRVT_OK;
}
