// Structured hierarchical layout (Sec. 3.2.4 "Data Reduction and Structured
// Data Layout", Fig. 5): the voxels that lie in a cell, ordered by band, then
// component, then cell, then linear index, with offsets per cell, component
// and band, so that every feature of the hierarchy is one contiguous range.
//
// Cells are ordered by (component, site id): the sites are sorted stably by
// component with an LSD radix sort, and rank[s] is the position of site s.
// Components are numbered band-major, so this order is also band-major.
//
// Voxels are placed by a deterministic counting sort.  The volume is cut
// into tiles of 4096 consecutive linear indices.  One wave walks a tile in
// index order, 64 voxels at a time: ballots split each group into runs of
// equal cell, and an LDS hash table numbers the distinct cells of the tile
// in order of first appearance.  Every (tile, cell) pair becomes one segment
// of the output.  The pairs are sorted stably by cell rank, so the segments
// of a cell follow each other in tile order, and an exclusive scan of their
// sizes gives every segment's start.  A last walk writes each voxel to its
// segment start plus the number of earlier voxels of its cell in the tile.
// Tiles with more distinct cells than the common kernel's table holds are
// listed and walked with a medium table, and those that overflow it by a
// kernel whose table covers a whole tile.
#include "layout.h"

namespace lsrvt {

namespace {

// Three table sizes: tiles with at most 256 distinct cells (almost all) are
// walked with a small table, so many waves fit a CU; a tile with more is
// deferred to a medium table (640), and from there to one that covers a
// whole tile.
constexpr int kSmallCap = 512, kSmallMax = 256;
constexpr int kMidCap = 1024, kMidMax = 640;
constexpr int kBigCap = kLayTile, kBigMax = kLayTile;
constexpr int kLayAhead = 4;  // 64-voxel groups whose cells are loaded ahead of the walk

enum { kPassCount = 0, kPassPairs = 1, kPassPlace = 2 };

template <int Cap, int MaxD>
struct TileTab {
  uint32_t key[Cap];    // cell id, kNone = empty
  uint32_t slot[Cap];   // order of first appearance in the tile
  uint32_t val[MaxD];   // per slot: running voxel count or next output index
};

struct LayArgs {
  const uint32_t *cell;
  int64_t n;
  uint32_t S;
  int64_t n_tiles;
  unsigned long long *cnt;
  uint32_t *tile_nd;
  uint8_t *tile_big;    // 0: small table, 1: medium, 2: whole-tile table
  uint32_t *big_list;   // tiles deferred by the small table
  uint32_t *huge_list;  // tiles deferred by the medium table
  uint32_t *big_cnt;    // [0] big_list length, [1] huge_list length
  const uint32_t *pair_off;
  uint32_t *pair_cell, *pair_cnt;
  const uint32_t *seg_off;
  uint32_t *perm;
};

// One wave walks one tile, 64 voxels at a time, with the cells of the next
// kLayAhead groups loaded while the current ones are walked.  Returns false
// (and has no side effects in the count and pair passes) when the tile has
// more than MaxD distinct cells.
template <int Cap, int MaxD, int Pass>
__device__ bool lay_walk(const LayArgs &A, int64_t tile, TileTab<Cap, MaxD> &T, uint32_t &nd_out) {
  const int lane = threadIdx.x;
  for (int i = lane; i < Cap; i += kWave) T.key[i] = kNone;
  const int64_t v0 = tile * kLayTile;
  if (Pass == kPassPlace) {
    // segment starts of the tile's pairs, in the same first-appearance order
    const uint32_t p0 = A.pair_off[tile], np = A.pair_off[tile + 1] - p0;
    for (uint32_t i = lane; i < np && i < (uint32_t)MaxD; i += kWave) T.val[i] = A.seg_off[p0 + i];
  }
  __syncthreads();
  auto load = [&](int g) {
    const int64_t v = v0 + g + lane;
    const uint32_t c = v < A.n ? A.cell[v] : kNone;
    return c < A.S ? c : kNone;
  };
  uint32_t cur[kLayAhead], nxt[kLayAhead];
#pragma unroll
  for (int j = 0; j < kLayAhead; ++j) cur[j] = load(j * kWave);
  uint32_t nd = 0, last_c = kNone, last_s = 0;
  for (int g0 = 0; g0 < kLayTile; g0 += kLayAhead * kWave) {
    if (g0 + kLayAhead * kWave < kLayTile) {
#pragma unroll
      for (int j = 0; j < kLayAhead; ++j) nxt[j] = load(g0 + (kLayAhead + j) * kWave);
    }
#pragma unroll
    for (int j = 0; j < kLayAhead; ++j) {
      const int g = g0 + j * kWave;
      const uint32_t c = cur[j];
      uint64_t rem = __ballot(c != kNone);
      while (rem) {
        const int leader = __ffsll((unsigned long long)rem) - 1;
        const uint32_t cl = __builtin_amdgcn_readlane(c, leader);
        const uint64_t mask = __ballot(c == cl);
        rem &= ~mask;
        uint32_t sl = last_s;
        if (cl != last_c) {
          uint32_t h = (cl * 2654435761u) & (Cap - 1);
          for (int probe = 0;; ++probe) {
            if (probe == Cap) return false;  // unreachable: the table always keeps a free slot for a new cell
            const uint32_t k = T.key[h];
            if (k == cl) {
              sl = T.slot[h];
              break;
            }
            if (k == kNone) {
              if (nd >= (uint32_t)MaxD) return false;
              // every lane stores the same values, so each lane reads back its own stores
              T.key[h] = cl;
              T.slot[h] = nd;
              sl = nd;
              if (Pass != kPassPlace) T.val[sl] = 0u;
              ++nd;
              break;
            }
            h = (h + 1) & (Cap - 1);
          }
          last_c = cl;
          last_s = sl;
        }
        const uint32_t base = T.val[sl];
        if (Pass == kPassPlace && ((mask >> lane) & 1ull))
          A.perm[base + (uint32_t)__popcll(mask & lanemask_lt())] = (uint32_t)(v0 + g + lane);
        T.val[sl] = base + (uint32_t)__popcll(mask);
      }
    }
#pragma unroll
    for (int j = 0; j < kLayAhead; ++j) cur[j] = nxt[j];
  }
  nd_out = nd;
  return true;
}

// Level 0 (small table) defers a tile to big_list, level 1 (medium) to
// huge_list; level 2 cannot fail.  Only the count pass defers; the later
// passes skip deferred tiles up front.
template <int Cap, int MaxD, int Pass, int Level>
__device__ void lay_tile(const LayArgs &A, int64_t tile, TileTab<Cap, MaxD> &T) {
  uint32_t nd = 0;
  const bool ok = lay_walk<Cap, MaxD, Pass>(A, tile, T, nd);
  __syncthreads();
  if (!ok) {
    if (Pass == kPassCount && Level < 2 && threadIdx.x == 0) {
      A.tile_big[tile] = (uint8_t)(Level + 1);
      A.tile_nd[tile] = 0;
      if (Level == 0) A.big_list[atomicAdd(&A.big_cnt[0], 1u)] = (uint32_t)tile;
      else A.huge_list[atomicAdd(&A.big_cnt[1], 1u)] = (uint32_t)tile;
    }
    return;
  }
  if (Pass == kPassCount) {
    for (int i = threadIdx.x; i < Cap; i += kWave) {
      const uint32_t k = T.key[i];
      if (k != kNone) atomicAdd(&A.cnt[k], (unsigned long long)T.val[T.slot[i]]);
    }
    if (threadIdx.x == 0) {
      A.tile_nd[tile] = nd;
      A.tile_big[tile] = (uint8_t)Level;
    }
  } else if (Pass == kPassPairs) {
    const uint32_t p0 = A.pair_off[tile];
    for (int i = threadIdx.x; i < Cap; i += kWave) {
      const uint32_t k = T.key[i];
      if (k != kNone) {
        A.pair_cell[p0 + T.slot[i]] = k;
        A.pair_cnt[p0 + T.slot[i]] = T.val[T.slot[i]];
      }
    }
  }
}

template <int Pass>
__global__ __launch_bounds__(kWave) void k_lay_small(LayArgs A) {
  __shared__ TileTab<kSmallCap, kSmallMax> T;
  for (int64_t tile = blockIdx.x; tile < A.n_tiles; tile += gridDim.x) {
    if (Pass != kPassCount && A.tile_big[tile]) continue;
    lay_tile<kSmallCap, kSmallMax, Pass, 0>(A, tile, T);
    __syncthreads();
  }
}

template <int Pass>
__global__ __launch_bounds__(kWave) void k_lay_mid(LayArgs A) {
  __shared__ TileTab<kMidCap, kMidMax> T;
  const uint32_t nb = A.big_cnt[0];
  for (uint32_t i = blockIdx.x; i < nb; i += gridDim.x) {
    const uint32_t tile = A.big_list[i];
    if (Pass != kPassCount && A.tile_big[tile] != 1) continue;
    lay_tile<kMidCap, kMidMax, Pass, 1>(A, tile, T);
    __syncthreads();
  }
}

template <int Pass>
__global__ __launch_bounds__(kWave) void k_lay_big(LayArgs A) {
  __shared__ TileTab<kBigCap, kBigMax> T;
  const uint32_t nb = A.big_cnt[1];
  for (uint32_t i = blockIdx.x; i < nb; i += gridDim.x) {
    lay_tile<kBigCap, kBigMax, Pass, 2>(A, A.huge_list[i], T);
    __syncthreads();
  }
}

// ---- small helpers ---------------------------------------------------------
__global__ void k_iota32(uint32_t *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (uint32_t)i;
}
// dst[pos[i]] = src[i]
__global__ void k_scatter32(const uint32_t *src, const uint32_t *pos, int64_t n, uint32_t *dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[pos[i]] = src[i];
}
// dst[i] = src[idx[i]]
__global__ void k_gather32(const uint32_t *src, const uint32_t *idx, int64_t n, uint32_t *dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}

// site sort: key = min(site_comp, C) (out-of-range components last)
__global__ void k_site_count(const uint32_t *site_comp, uint32_t S, uint32_t C, uint32_t *ccount) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < S) atomicAdd(&ccount[min(site_comp[i], C)], 1u);
}
__global__ void k_site_digit(const uint32_t *val, uint32_t S, const uint32_t *site_comp, uint32_t C, int shift,
                             uint8_t *digit) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < S) digit[i] = (uint8_t)(min(site_comp[val[i]], C) >> shift);
}
__global__ void k_site_rank(const uint32_t *order, uint32_t S, uint32_t *rank) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < S) rank[order[i]] = i;
}
__global__ void k_pair_digit(const uint32_t *val, int64_t P, const uint32_t *pair_cell, const uint32_t *rank,
                             int shift, uint8_t *digit) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < P) digit[i] = (uint8_t)(rank[pair_cell[val[i]]] >> shift);
}
__global__ void k_cnt_rank(const unsigned long long *cnt, const uint32_t *order, uint32_t S, uint32_t *cnt_rank) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < S) cnt_rank[i] = (uint32_t)cnt[order[i]];
}

int bits_for(uint64_t maxval) {
  int b = 0;
  while (b < 64 && (maxval >> b) != 0) ++b;
  return b;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

}  // namespace

size_t layout_scratch(const Geom &g, uint32_t S, uint32_t C) {
  const int64_t P = layout_pair_cap(g, S);
  const int64_t T = layout_tiles(g);
  int64_t m = P > (int64_t)S ? P : (int64_t)S;
  if (m < (int64_t)C + 3) m = (int64_t)C + 3;
  if (m < T + 1) m = T + 1;
  size_t a = StableSort8::workspace(m);
  size_t b = ScanU32::workspace(m + 1);
  return (a > b ? a : b) + 256;
}

int32_t layout_sites(const uint32_t *site_comp, uint32_t S, uint32_t C, LayoutWork &W, hipStream_t s) {
  int32_t rc;
  if ((rc = fill<uint32_t>(W.ccount, (int64_t)C + 2, 0u, s))) return rc;
  if (S) {
    hipLaunchKernelGGL(k_site_count, dim3(blocks_for(S)), dim3(256), 0, s, site_comp, S, C, W.ccount);
    hipLaunchKernelGGL(k_iota32, dim3(blocks_for(S)), dim3(256), 0, s, W.order, (int64_t)S);
    LSRVT_LAUNCHED();
    const int passes = (bits_for(C) + 7) / 8;
    uint32_t *cur = W.order, *other = W.sval;
    for (int p = 0; p < passes; ++p) {
      hipLaunchKernelGGL(k_site_digit, dim3(blocks_for(S)), dim3(256), 0, s, cur, S, site_comp, C, 8 * p, W.sdigit);
      LSRVT_LAUNCHED();
      if ((rc = StableSort8::run(W.sdigit, S, W.spos, nullptr, W.scratch, W.scratch_bytes, s))) return rc;
      hipLaunchKernelGGL(k_scatter32, dim3(blocks_for(S)), dim3(256), 0, s, cur, W.spos, (int64_t)S, other);
      LSRVT_LAUNCHED();
      uint32_t *t = cur;
      cur = other;
      other = t;
    }
    if (cur != W.order) {
      LSRVT_HIP(hipMemcpyAsync(W.order, cur, sizeof(uint32_t) * S, hipMemcpyDeviceToDevice, s));
    }
    hipLaunchKernelGGL(k_site_rank, dim3(blocks_for(S)), dim3(256), 0, s, W.order, S, W.rank);
    LSRVT_LAUNCHED();
  }
  return ScanU32::run(W.ccount, (int64_t)C + 2, W.coff, W.scratch, W.scratch_bytes, s);
}

int32_t layout_voxels(const uint32_t *cell, const Geom &g, uint32_t S, LayoutWork &W, uint32_t *perm, hipStream_t s) {
  int32_t rc;
  if ((rc = fill<unsigned long long>(W.cnt, S ? S : 1, 0ull, s))) return rc;
  if ((rc = fill<uint32_t>(W.big_cnt, 2, 0u, s))) return rc;
  if (S == 0) return fill<uint32_t>(W.cell_off, 1, 0u, s);
  const int64_t T = W.n_tiles;
  LayArgs A;
  A.cell = cell;
  A.n = g.n;
  A.S = S;
  A.n_tiles = T;
  A.cnt = W.cnt;
  A.tile_nd = W.tile_nd;
  A.tile_big = W.tile_big;
  A.big_list = W.big_list;
  A.huge_list = W.huge_list;
  A.big_cnt = W.big_cnt;
  A.pair_off = W.pair_off;
  A.pair_cell = W.pair_cell;
  A.pair_cnt = W.pair_cnt;
  A.seg_off = W.pair_cnt;  // segment starts replace the counts before the place pass
  A.perm = perm;
  const unsigned grid = (unsigned)(T < 65535 ? T : 65535);
  const unsigned grid_mid = 2048, grid_big = 256;
  // 1. distinct cells per tile and voxels per site
  hipLaunchKernelGGL(k_lay_small<kPassCount>, dim3(grid), dim3(kWave), 0, s, A);
  hipLaunchKernelGGL(k_lay_mid<kPassCount>, dim3(grid_mid), dim3(kWave), 0, s, A);
  hipLaunchKernelGGL(k_lay_big<kPassCount>, dim3(grid_big), dim3(kWave), 0, s, A);
  LSRVT_LAUNCHED();
  if ((rc = ScanU32::run(W.tile_nd, T, W.pair_off, W.scratch, W.scratch_bytes, s))) return rc;
  uint32_t P = 0;
  {
    const int32_t rc_ = read_words(W.pair_off + T, 1, &P, s);
    if (rc_) return rc_;
  }
  if ((int64_t)P > W.pair_cap) return LSRVT_EDEVICE;  // cannot happen: the capacity is an upper bound
  // 2. the pairs, in tile order
  hipLaunchKernelGGL(k_lay_small<kPassPairs>, dim3(grid), dim3(kWave), 0, s, A);
  hipLaunchKernelGGL(k_lay_mid<kPassPairs>, dim3(grid_mid), dim3(kWave), 0, s, A);
  hipLaunchKernelGGL(k_lay_big<kPassPairs>, dim3(grid_big), dim3(kWave), 0, s, A);
  LSRVT_LAUNCHED();
  // 3. stable sort of the pairs by cell rank
  if (P) {
    hipLaunchKernelGGL(k_iota32, dim3(blocks_for(P)), dim3(256), 0, s, W.val_a, (int64_t)P);
    LSRVT_LAUNCHED();
    const int passes = (bits_for(S - 1) + 7) / 8;
    uint32_t *cur = W.val_a, *other = W.val_b;
    for (int p = 0; p < passes; ++p) {
      hipLaunchKernelGGL(k_pair_digit, dim3(blocks_for(P)), dim3(256), 0, s, cur, (int64_t)P, W.pair_cell, W.rank,
                         8 * p, W.digit);
      LSRVT_LAUNCHED();
      if ((rc = StableSort8::run(W.digit, P, W.pos, nullptr, W.scratch, W.scratch_bytes, s))) return rc;
      hipLaunchKernelGGL(k_scatter32, dim3(blocks_for(P)), dim3(256), 0, s, cur, W.pos, (int64_t)P, other);
      LSRVT_LAUNCHED();
      uint32_t *t = cur;
      cur = other;
      other = t;
    }
    // 4. segment starts: scan the sizes in sorted order, scatter back to pair order
    hipLaunchKernelGGL(k_gather32, dim3(blocks_for(P)), dim3(256), 0, s, W.pair_cnt, cur, (int64_t)P, W.pos);
    LSRVT_LAUNCHED();
    if ((rc = ScanU32::run(W.pos, P, other, W.scratch, W.scratch_bytes, s))) return rc;
    hipLaunchKernelGGL(k_scatter32, dim3(blocks_for(P)), dim3(256), 0, s, other, cur, (int64_t)P, W.pair_cnt);
    LSRVT_LAUNCHED();
    // 5. place every voxel
    hipLaunchKernelGGL(k_lay_small<kPassPlace>, dim3(grid), dim3(kWave), 0, s, A);
    hipLaunchKernelGGL(k_lay_mid<kPassPlace>, dim3(grid_mid), dim3(kWave), 0, s, A);
    hipLaunchKernelGGL(k_lay_big<kPassPlace>, dim3(grid_big), dim3(kWave), 0, s, A);
    LSRVT_LAUNCHED();
  }
  // cell offsets by rank
  hipLaunchKernelGGL(k_cnt_rank, dim3(blocks_for(S)), dim3(256), 0, s, W.cnt, W.order, S, W.cnt_rank);
  LSRVT_LAUNCHED();
  return ScanU32::run(W.cnt_rank, S, W.cell_off, W.scratch, W.scratch_bytes, s);
}

namespace {

// comp_off[c] = cell_off[coff[c]] for c <= C
__global__ void k_comp_off(const uint32_t *cell_off, const uint32_t *coff, uint32_t C, uint32_t *comp_off) {
  uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c <= C) comp_off[c] = cell_off[coff[c]];
}
// band_off[b] = comp_off[first component whose band is >= b] (bands nondecreasing in component id)
__global__ void k_band_off(const uint8_t *comp_band, uint32_t C, int32_t n_bands, const uint32_t *comp_off,
                           uint32_t *band_off) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b > n_bands) return;
  uint32_t lo = 0, hi = C;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if ((int)comp_band[mid] < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  band_off[b] = comp_off[lo];
}

// out[j][k] = vars[j][perm[k]]
__global__ void k_extract(const float *__restrict__ vars, int64_t n, int m, const uint32_t *__restrict__ perm,
                          int64_t count, float *__restrict__ out) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const int64_t v = perm[k];
  for (int j = 0; j < m; ++j) out[(int64_t)j * count + k] = v < n ? vars[(int64_t)j * n + v] : __builtin_nanf("");
}

struct LaySizer : Sizer {
  template <class T>
  T *take(size_t c) {
    Sizer::take<T>(c);
    return nullptr;
  }
};

}  // namespace

}  // namespace lsrvt

using namespace lsrvt;

extern "C" size_t lsrvt_layout_workspace(lsrvt_dims dims, uint32_t n_sites, uint32_t n_comp) {
  Geom g;
  if (make_geom(dims, g)) return 0;
  LaySizer z;
  layout_take(z, g, n_sites, n_comp, nullptr);
  return z.off + layout_scratch(g, n_sites, n_comp);
}

extern "C" int32_t lsrvt_layout(const uint32_t *d_cell, lsrvt_dims dims, const uint32_t *d_site_comp, uint32_t n_sites,
                                const uint8_t *d_comp_band, uint32_t n_comp, int32_t n_bands, uint32_t *d_perm,
                                uint32_t *d_site_order, uint32_t *d_cell_off, uint32_t *d_comp_off,
                                uint32_t *d_band_off, uint32_t *h_n_placed, void *d_work, size_t work_bytes,
                                void *stream) {
  Geom g;
  int32_t rc = make_geom(dims, g);
  if (rc) return rc;
  if (n_bands < 1 || n_bands > 255) return LSRVT_EINVAL;
  if (!d_cell || !d_perm || !d_cell_off || !d_comp_off || !d_band_off) return LSRVT_EINVAL;
  if (n_sites && (!d_site_comp || !d_site_order)) return LSRVT_EINVAL;
  if (n_comp && !d_comp_band) return LSRVT_EINVAL;
  if ((rc = check_work(d_work, work_bytes, lsrvt_layout_workspace(dims, n_sites, n_comp)))) return rc;
  Carve cv(d_work, work_bytes);
  LayoutWork W;
  layout_take(cv, g, n_sites, n_comp, &W);
  if (!cv.ok) return LSRVT_EWORKSPACE;
  W.scratch = cv.base + cv.off;
  W.scratch_bytes = cv.size - cv.off;
  hipStream_t s = as_stream(stream);
  if ((rc = layout_sites(d_site_comp, n_sites, n_comp, W, s))) return rc;
  if ((rc = layout_voxels(d_cell, g, n_sites, W, d_perm, s))) return rc;
  if (n_sites) {
    LSRVT_HIP(hipMemcpyAsync(d_site_order, W.order, sizeof(uint32_t) * n_sites, hipMemcpyDeviceToDevice, s));
  }
  LSRVT_HIP(hipMemcpyAsync(d_cell_off, W.cell_off, sizeof(uint32_t) * ((size_t)n_sites + 1), hipMemcpyDeviceToDevice,
                           s));
  hipLaunchKernelGGL(k_comp_off, dim3(blocks_for((int64_t)n_comp + 1)), dim3(256), 0, s, W.cell_off, W.coff, n_comp,
                     d_comp_off);
  hipLaunchKernelGGL(k_band_off, dim3(blocks_for(n_bands + 1)), dim3(256), 0, s, d_comp_band, n_comp, n_bands,
                     d_comp_off, d_band_off);
  LSRVT_LAUNCHED();
  uint32_t placed = 0;
  {
    const int32_t rc_ = read_words(W.cell_off + n_sites, 1, &placed, s);
    if (rc_) return rc_;
  }
  if (h_n_placed) *h_n_placed = placed;
  return LSRVT_OK;
}

extern "C" int32_t lsrvt_extract(const float *d_vars, int32_t n_vars, lsrvt_dims dims, const uint32_t *d_perm,
                                 uint32_t n_placed, float *d_out, void *stream) {
  Geom g;
  int32_t rc = make_geom(dims, g);
  if (rc) return rc;
  if (n_vars < 1 || (int64_t)n_placed > g.n) return LSRVT_EINVAL;
  if (n_placed == 0) return LSRVT_OK;
  if (!d_vars || !d_perm || !d_out) return LSRVT_EINVAL;
  hipLaunchKernelGGL(k_extract, dim3(blocks_for(n_placed)), dim3(256), 0, as_stream(stream), d_vars, g.n, n_vars,
                     d_perm, (int64_t)n_placed, d_out);
  LSRVT_LAUNCHED();
  return LSRVT_OK;
}
