// Structured hierarchical layout (Sec. 3.2.4, Fig. 5): internal interface
// shared by the statistics pipeline and the layout entry point.
#pragma once

#include "common.h"

namespace lsrvt {

constexpr int kLayTile = 4096;  // consecutive linear indices walked by one wave

// Device buffers of one layout build.  Cells are numbered by rank: the
// position of their site when sites are sorted stably by component.
struct LayoutWork {
  // sites
  uint32_t *order;   // [S] site ids in (component, id) order
  uint32_t *rank;    // [S] inverse of order
  uint32_t *ccount;  // [C + 2] sites per component (last slot: site_comp >= C)
  uint32_t *coff;    // [C + 3] exclusive offsets of ccount
  uint32_t *sval;    // [S] radix-sort ping-pong
  uint8_t *sdigit;   // [S]
  uint32_t *spos;    // [S]
  // voxels
  unsigned long long *cnt;  // [S] voxels per site
  uint32_t *cnt_rank;       // [S] voxels per cell, by rank
  uint32_t *cell_off;       // [S + 1] start of every cell, by rank
  uint32_t *tile_nd;        // [T] distinct cells per tile
  uint32_t *pair_off;       // [T + 1] first (tile, cell) pair of every tile
  uint8_t *tile_big;        // [T] 0: small table, 1: medium table, 2: whole-tile table
  uint32_t *big_list;       // [T] tiles deferred by the small table
  uint32_t *huge_list;      // [T] tiles deferred by the medium table
  uint32_t *big_cnt;        // [4] [0] big_list length, [1] huge_list length
  uint32_t *pair_cell;      // [Pcap] cell of every pair, then reused
  uint32_t *pair_cnt;       // [Pcap] voxels of every pair, then segment starts
  uint32_t *val_a, *val_b;  // [Pcap + 1] pair sort ping-pong / scan output
  uint32_t *pos;            // [Pcap + 1]
  uint8_t *digit;           // [Pcap]
  int64_t n_tiles, pair_cap;
  void *scratch;  // ScanU32 / StableSort8 scratch
  size_t scratch_bytes;
};

inline int64_t layout_tiles(const Geom &g) { return (g.n + kLayTile - 1) / kLayTile; }

// Exact bound on the number of (tile, cell) pairs: at most one per voxel and
// at most min(S, tile size) per tile.
inline int64_t layout_pair_cap(const Geom &g, uint32_t S) {
  const int64_t T = layout_tiles(g);
  const int64_t per = S < (uint32_t)kLayTile ? (int64_t)S : (int64_t)kLayTile;
  const int64_t a = T * per;
  return (a < g.n ? a : g.n) + 1;
}

template <class A>
void layout_take(A &a, const Geom &g, uint32_t S, uint32_t C, LayoutWork *W) {
  const size_t s1 = S ? S : 1;
  const int64_t T = layout_tiles(g);
  const int64_t P = layout_pair_cap(g, S);
  auto order = a.template take<uint32_t>(s1);
  auto rank = a.template take<uint32_t>(s1);
  auto ccount = a.template take<uint32_t>((size_t)C + 2);
  auto coff = a.template take<uint32_t>((size_t)C + 3);
  auto sval = a.template take<uint32_t>(s1);
  auto sdigit = a.template take<uint8_t>(s1);
  auto spos = a.template take<uint32_t>(s1);
  auto cnt = a.template take<unsigned long long>(s1);
  auto cnt_rank = a.template take<uint32_t>(s1);
  auto cell_off = a.template take<uint32_t>(s1 + 1);
  auto tile_nd = a.template take<uint32_t>(T);
  auto pair_off = a.template take<uint32_t>(T + 1);
  auto tile_big = a.template take<uint8_t>(T);
  auto big_list = a.template take<uint32_t>(T);
  auto huge_list = a.template take<uint32_t>(T);
  auto big_cnt = a.template take<uint32_t>(4);
  auto pair_cell = a.template take<uint32_t>(P);
  auto pair_cnt = a.template take<uint32_t>(P);
  auto val_a = a.template take<uint32_t>(P + 1);
  auto val_b = a.template take<uint32_t>(P + 1);
  auto pos = a.template take<uint32_t>(P + 1);
  auto digit = a.template take<uint8_t>(P);
  if (W) {
    W->order = order;
    W->rank = rank;
    W->ccount = ccount;
    W->coff = coff;
    W->sval = sval;
    W->sdigit = sdigit;
    W->spos = spos;
    W->cnt = cnt;
    W->cnt_rank = cnt_rank;
    W->cell_off = cell_off;
    W->tile_nd = tile_nd;
    W->pair_off = pair_off;
    W->tile_big = tile_big;
    W->big_list = big_list;
    W->huge_list = huge_list;
    W->big_cnt = big_cnt;
    W->pair_cell = pair_cell;
    W->pair_cnt = pair_cnt;
    W->val_a = val_a;
    W->val_b = val_b;
    W->pos = pos;
    W->digit = digit;
    W->n_tiles = T;
    W->pair_cap = P;
  }
}

// Scratch needed by the scans and sorts of a layout build.
size_t layout_scratch(const Geom &g, uint32_t S, uint32_t C);

// Sites sorted stably by component: order, rank, ccount, coff.
int32_t layout_sites(const uint32_t *site_comp, uint32_t S, uint32_t C, LayoutWork &W, hipStream_t s);

// Voxel counts per site, cell offsets by rank and the voxel permutation
// (perm[cell_off[r] ...] = voxels of the cell of rank r in index order).
// Needs layout_sites first.
int32_t layout_voxels(const uint32_t *cell, const Geom &g, uint32_t S, LayoutWork &W, uint32_t *perm, hipStream_t s);

}  // namespace lsrvt
