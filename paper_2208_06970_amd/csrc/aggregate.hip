// Statistics of every cell, merged cell -> component -> band (Sec. 3.3,
// "Aggregation"; the hierarchy of Sec. 3.2.4 / Fig. 5).
//
// Pipeline:
//  1. the structured layout (layout.hip) lists the voxels of every cell as
//     one contiguous range, cells in (component, site id) order and voxels
//     in index order;
//  2. every cell's range is cut into work items of at most kItemVoxels;
//  3. one workgroup per item gathers the item's values into LDS, shifted by
//     the value at the cell's site, and accumulates per "unit" float32 sums
//     with an error-free two-sum compensation (hi + lo): units are sum d_j
//     and sum d_j d_k (the product error of d_j d_k is folded into lo with
//     an FMA).  Lanes own units, so the order of every sum is fixed.
//     Histograms and extrema are integer / compare operations and go through
//     LDS and then global atomics;
//  4. per cell, the item partials are combined in item order; the
//     compensated float32 pair of every unit is exact in float64, where the
//     cell's mean, M2 and co-moments are formed once (a constant amount of
//     work per cell, and the inputs the float64 merges need); the float32
//     cell outputs are those values rounded once.  Every sum over voxels is
//     float32;
//  5. Chan et al.'s pairwise merge in float64: cells of a component in site
//     id order, then components of a band in component id order.  Counts,
//     extrema and histograms merge exactly with atomics.
#include <algorithm>

#include "layout.h"

namespace lsrvt {

namespace {

constexpr int kAggThreads = 256;
constexpr int kAggMaxThreads = 512;  // k_agg_cell with two lane groups of up to 256 units
constexpr int kMaxVars = 32;
constexpr int kMaxPairs = kMaxVars * (kMaxVars + 1) / 2;
constexpr int64_t kItemVoxels = 4096;
constexpr int kSmallCell = 256;  // cells up to this size are summed by a single wave
constexpr int kMaxHist = 8192;  // n_vars * n_bins

struct Pairs {
  uint8_t j[kMaxPairs];
  uint8_t k[kMaxPairs];
};

struct BBox {
  uint32_t *x0, *x1, *y0, *y1, *z0, *z1;
};

__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
  s = a + b;
  float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Compensated accumulate of x (with an exact extra error term ex) into (hi, lo).
__device__ __forceinline__ void acc(float &hi, float &lo, float x, float ex) {
  float s, e;
  two_sum(hi, x, s, e);
  hi = s;
  lo += e + ex;
}

// ---------------------------------------------------------------------------
// 1-2. the voxels of every cell are a contiguous range of the structured
// layout (layout.hip); each cell's range is cut into items of at most
// kItemVoxels voxels, numbered in cell rank order.
__global__ void k_agg_items(const uint32_t *__restrict__ cnt_rank, uint32_t S, uint32_t *items) {
  uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < S) items[r] = (uint32_t)((cnt_rank[r] + kItemVoxels - 1) / kItemVoxels);
}

// item -> cell rank, and the split into cells small enough for one wave
// (their single item) and the items of larger cells
__global__ void k_item_cells(const uint32_t *__restrict__ item_off, const uint32_t *__restrict__ cnt_rank, uint32_t S,
                             int small_ok, uint32_t *item_rank, uint32_t *small_list, uint32_t *big_list,
                             uint32_t *counts) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = r < S;
  const uint32_t i0 = in ? item_off[r] : 0u, i1 = in ? item_off[r + 1] : 0u;
  const bool small = in && small_ok && cnt_rank[r] <= (uint32_t)kSmallCell;
  const uint32_t n = i1 - i0;
  // one counter atomic per wave and list: wave prefix sums of the item counts
  const int lane = lane_id();
  uint32_t ns = small ? n : 0u, nb = small ? 0u : n;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t a = __shfl_up(ns, o, kWave), b = __shfl_up(nb, o, kWave);
    if (lane >= o) {
      ns += a;
      nb += b;
    }
  }
  const uint32_t ts = __shfl(ns, kWave - 1, kWave), tb = __shfl(nb, kWave - 1, kWave);
  uint32_t bs = 0, bb = 0;
  if (lane == 0) {
    if (ts) bs = atomicAdd(&counts[0], ts);
    if (tb) bb = atomicAdd(&counts[1], tb);
  }
  bs = __shfl(bs, 0, kWave);
  bb = __shfl(bb, 0, kWave);
  const uint32_t p = small ? bs + ns - n : bb + nb - n;
  for (uint32_t i = i0; i < i1; ++i) {
    item_rank[i] = r;
    (small ? small_list : big_list)[p + (i - i0)] = i;
  }
}

// 3. per-item compensated sums
struct CellArgs {
  const uint32_t *perm;       // layout order of the voxels
  const uint32_t *cell_off;   // [S + 1] by rank
  const uint32_t *order;      // rank -> site
  const uint32_t *sites;
  const float *vars;  // [m][N]
  const float *edges; // [m][B+1] or null
  int64_t n;
  int m, B, U, G, P, tile;  // tile: voxels staged in LDS per round (1, 2 or 4 times the block size)
  Pairs pairs;
  const uint32_t *item_off;   // [S + 1] by rank
  const uint32_t *item_rank;  // [n_items]
  const uint32_t *list;       // items of this launch
  const uint32_t *list_cnt;   // their number (device)
  float *part_hi, *part_lo;  // [n_items][U]
  uint32_t *hist;            // cell histograms [S][m][B] (zeroed) or null
  uint32_t *kmin, *kmax;     // ordered keys [S][m]
};

constexpr int kMaxVPT = 4;  // voxels per thread and round

// Wave-wide min / max by DPP lane moves (quad permutes, row mirrors, row
// broadcasts; every lane of the wave active): the result is read from the
// last lane and returned to all lanes.
#define LSRVT_DPP_STEP(OP, ID, CTRL, RMASK) \
  v = OP(v, (uint32_t)__builtin_amdgcn_update_dpp((int)(ID), (int)v, CTRL, RMASK, 0xF, false))
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  LSRVT_DPP_STEP(min, 0xFFFFFFFFu, 0xB1, 0xF);   // quad_perm [1,0,3,2]
  LSRVT_DPP_STEP(min, 0xFFFFFFFFu, 0x4E, 0xF);   // quad_perm [2,3,0,1]
  LSRVT_DPP_STEP(min, 0xFFFFFFFFu, 0x141, 0xF);  // row_half_mirror
  LSRVT_DPP_STEP(min, 0xFFFFFFFFu, 0x140, 0xF);  // row_mirror
  LSRVT_DPP_STEP(min, 0xFFFFFFFFu, 0x142, 0xA);  // row_bcast:15 into rows 1 and 3
  LSRVT_DPP_STEP(min, 0xFFFFFFFFu, 0x143, 0xC);  // row_bcast:31 into rows 2 and 3
  return (uint32_t)__builtin_amdgcn_readlane((int)v, kWave - 1);
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  LSRVT_DPP_STEP(max, 0u, 0xB1, 0xF);
  LSRVT_DPP_STEP(max, 0u, 0x4E, 0xF);
  LSRVT_DPP_STEP(max, 0u, 0x141, 0xF);
  LSRVT_DPP_STEP(max, 0u, 0x140, 0xF);
  LSRVT_DPP_STEP(max, 0u, 0x142, 0xA);
  LSRVT_DPP_STEP(max, 0u, 0x143, 0xC);
  return (uint32_t)__builtin_amdgcn_readlane((int)v, kWave - 1);
}
#undef LSRVT_DPP_STEP

// Histogram bin of x: #{interior edges e_1..e_{B-1} <= x} for ascending
// edges e_0..e_B (sc = B / (e_B - e_0)).  A guess from the mean edge spacing
// is kept when the two edges around it confirm it (always, for evenly spaced
// edges); otherwise bisection.  NaN lands in bin 0, as every comparison with
// it is false.
__device__ __forceinline__ int hist_bin(float x, const float *e, int B, float e0, float sc) {
  const int g = (int)fminf(fmaxf((x - e0) * sc, 0.0f), (float)(B - 1));
  if ((g == 0 || e[g] <= x) && (g == B - 1 || x < e[g + 1])) return g;
  int a = 1, b = B;
  while (a < b) {
    const int mid = (a + b) >> 1;
    if (e[mid] <= x)
      a = mid + 1;
    else
      b = mid;
  }
  return a - 1;
}

// R = unit slots per lane: with R == 1 the U units are replicated over G
// lane groups that split each staging round's voxels into G contiguous
// ranges (multiples of four voxels, in order; the workgroup has at least
// G * U threads); with R > 1 (more units than lanes) lane t owns units t,
// t + NT, ... and G = 1.  VPT = voxels staged per thread and round (the
// round holds VPT * NT voxels).
template <int R, int VPT>
__global__ __launch_bounds__(kAggMaxThreads) void k_agg_cell(CellArgs A) {
  extern __shared__ uint8_t smem[];
  const int m = A.m, B = A.B, U = A.U, G = A.G, TL = A.tile, ld = A.tile + 4;
  const int NT = blockDim.x;
  float *dv = reinterpret_cast<float *>(smem);                       // [m][TL + 4] values minus the site value
  float *ones = dv + m * ld;                                         // [TL + 4] 1.0: the second factor of Σd
  uint32_t *hist_l = reinterpret_cast<uint32_t *>(ones + ld);        // [m*B]
  uint32_t *kmin_l = hist_l + m * B;                                 // [m]
  uint32_t *kmax_l = kmin_l + m;                                     // [m]
  float *K = reinterpret_cast<float *>(kmax_l + m);                  // [m]
  float *ph = K + m;                                                 // [G*U]
  float *pl = ph + G * U;                                            // [G*U]
  float *edg = pl + G * U;                                           // [m][B+1]
  float *scl = edg + m * (B + 1);                                    // [m] B / (e_B - e_0)
  const int t = threadIdx.x;
  const int lane = lane_id();
  const int grp = R == 1 ? t / U : 0;
  if (B > 0) {
    for (int i = t; i < m * (B + 1); i += NT) edg[i] = A.edges[i];
    for (int j = t; j < m; j += NT) scl[j] = (float)B / (A.edges[j * (B + 1) + B] - A.edges[j * (B + 1)]);
  }
  for (int i = t; i < ld; i += NT) ones[i] = 1.0f;

  const uint32_t n_list = *A.list_cnt;
  for (uint32_t k = blockIdx.x; k < n_list; k += gridDim.x) {
    const uint32_t item = A.list[k];
    const uint32_t r = A.item_rank[item];
    const uint32_t s = A.order[r];
    const uint32_t part = item - A.item_off[r];
    const uint32_t start = A.cell_off[r] + part * (uint32_t)kItemVoxels;
    const uint32_t stop = min(A.cell_off[r + 1], start + (uint32_t)kItemVoxels);

    for (int i = t; i < m * B; i += NT) hist_l[i] = 0;
    if (t < m) {
      kmin_l[t] = 0xFFFFFFFFu;
      kmax_l[t] = 0u;
      K[t] = A.vars[(int64_t)t * A.n + A.sites[s]];
    }
    float hi[R], lo[R];
#pragma unroll
    for (int q = 0; q < R; ++q) hi[q] = lo[q] = 0.0f;
    __syncthreads();

    for (uint32_t base = start; base < stop; base += (uint32_t)TL) {
      const int nt = (int)min((uint32_t)TL, stop - base);
      // stage: thread t owns voxels t, t + NT, ... of the round
      uint32_t vv[VPT];
      bool ok[VPT];
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        const int q = t + i * NT;
        ok[i] = q < nt;
        vv[i] = ok[i] ? A.perm[base + q] : 0u;
      }
#pragma unroll 2
      for (int j = 0; j < m; ++j) {
        const float kj = K[j];
        const float *col = A.vars + (int64_t)j * A.n;
        float x[VPT];
#pragma unroll
        for (int i = 0; i < VPT; ++i) x[i] = ok[i] ? col[vv[i]] : 0.0f;
        uint32_t kmn = 0xFFFFFFFFu, kmx = 0u;
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
          if (!ok[i]) continue;
          dv[j * ld + t + i * NT] = x[i] - kj;
          const uint32_t kk = f2key(x[i]);
          kmn = min(kmn, kk);
          kmx = max(kmx, kk);
        }
        kmn = wave_min_u32(kmn);
        kmx = wave_max_u32(kmx);
        if (lane == 0) {
          if (kmn != 0xFFFFFFFFu) atomicMin(&kmin_l[j], kmn);
          if (kmx != 0u) atomicMax(&kmax_l[j], kmx);
        }
        if (B > 0) {
          const float *e = edg + j * (B + 1);
          const float e0 = e[0], sc = scl[j];
#pragma unroll
          for (int i = 0; i < VPT; ++i)
            // one LDS atomic per lane; the LDS serialises lanes that hit one bin
            if (ok[i]) atomicAdd(&hist_l[j * B + hist_bin(x[i], e, B, e0, sc)], 1u);
        }
      }
      __syncthreads();
      // this group's voxels of the round: [v0, v1), four at a time
      const int cs = R == 1 ? ((nt + G - 1) / G + 3) & ~3 : nt;
      const int v0 = min(nt, grp * cs), v1 = min(nt, v0 + cs);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int u = R == 1 ? t % U : t + q * NT;
        const bool worker = R == 1 ? t < G * U : u < U;
        if (!worker) continue;
        // every unit sums products: Σd_j d_k, and Σd_j as d_j times a row of
        // ones (d·1 is d exactly and its product error 0, so the sum is the
        // one of d itself; only a d of ±inf, |x - x_site| beyond the float
        // range, would give NaN instead of ±inf), so the lanes of a wave
        // take one path
        const float *dj, *dk;
        if (u < m) {
          dj = dv + u * ld;
          dk = ones;
        } else {
          const int p = u - m;
          dj = dv + A.pairs.j[p] * ld;
          dk = dv + A.pairs.k[p] * ld;
        }
        int v = v0;
        for (; v + 4 <= v1; v += 4) {
          const float4 a = *reinterpret_cast<const float4 *>(dj + v);
          const float4 b = *reinterpret_cast<const float4 *>(dk + v);
          const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float pr = av[i] * bv[i];
            const float pe = __builtin_fmaf(av[i], bv[i], -pr);  // exact error of the product
            acc(hi[q], lo[q], pr, pe);
          }
        }
        for (; v < v1; ++v) {
          const float a0 = dj[v], b0 = dk[v];
          const float pr = a0 * b0;
          const float pe = __builtin_fmaf(a0, b0, -pr);
          acc(hi[q], lo[q], pr, pe);
        }
      }
      __syncthreads();
    }
    // combine the lane groups in group order
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int u = R == 1 ? t % U : t + q * NT;
      const bool worker = R == 1 ? t < G * U : u < U;
      if (worker) {
        ph[grp * U + u] = hi[q];
        pl[grp * U + u] = lo[q];
      }
    }
    __syncthreads();
    for (int u = t; u < U; u += NT) {
      float H = 0.0f, Lo = 0.0f;
      for (int gg = 0; gg < G; ++gg) {
        acc(H, Lo, ph[gg * U + u], 0.0f);
        Lo += pl[gg * U + u];
      }
      A.part_hi[(int64_t)item * U + u] = H;
      A.part_lo[(int64_t)item * U + u] = Lo;
    }
    // flush exact integer/compare statistics
    if (A.hist) {
      uint32_t *dst = A.hist + (int64_t)s * m * B;
      for (int i = t; i < m * B; i += NT)
        if (hist_l[i]) atomicAdd(&dst[i], hist_l[i]);
    }
    if (t < m) {
      if (kmin_l[t] != 0xFFFFFFFFu) atomicMin(&A.kmin[(int64_t)s * m + t], kmin_l[t]);
      if (kmax_l[t] != 0u) atomicMax(&A.kmax[(int64_t)s * m + t], kmax_l[t]);
    }
    __syncthreads();
  }
}

// The same sums for cells of at most kSmallCell voxels, one wave per cell:
// each wave has its own LDS region and synchronises only with itself.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__host__ __device__ inline size_t wave_region_words(int m, int B, int U, int G) {
  return (size_t)m * (kSmallCell + 1) + (size_t)m * B + 3 * (size_t)m + 2 * (size_t)G * U;
}

template <int R>
__global__ __launch_bounds__(kAggThreads) void k_agg_cell_wave(CellArgs A) {
  extern __shared__ uint8_t smem[];
  constexpr int kWaves = kAggThreads / kWave;
  constexpr int VPT = kSmallCell / kWave;
  const int m = A.m, B = A.B, U = A.U, G = A.G, ld = kSmallCell + 1;
  const int wid = threadIdx.x / kWave, lane = lane_id();
  float *edg = reinterpret_cast<float *>(smem);  // [m][B+1], shared by the waves
  float *ones = edg + m * (B + 1);               // [kSmallCell + 1] 1.0, shared: the second factor of Σd
  float *dv = ones + (kSmallCell + 1) + (size_t)wid * wave_region_words(m, B, U, G);
  uint32_t *hist_l = reinterpret_cast<uint32_t *>(dv + m * ld);  // [m*B]
  uint32_t *kmin_l = hist_l + m * B;
  uint32_t *kmax_l = kmin_l + m;
  float *K = reinterpret_cast<float *>(kmax_l + m);
  float *ph = K + m;
  float *pl = ph + G * U;
  const int grp = R == 1 ? lane / U : 0;
  if (B > 0)
    for (int i = threadIdx.x; i < m * (B + 1); i += kAggThreads) edg[i] = A.edges[i];
  for (int i = threadIdx.x; i < kSmallCell + 1; i += kAggThreads) ones[i] = 1.0f;
  __syncthreads();
  const uint32_t n_list = *A.list_cnt;
  for (uint32_t k = blockIdx.x * kWaves + wid; k < n_list; k += gridDim.x * kWaves) {
    const uint32_t item = A.list[k];
    const uint32_t r = A.item_rank[item];
    const uint32_t s = A.order[r];
    const uint32_t start = A.cell_off[r];
    const int nt = (int)(A.cell_off[r + 1] - start);
    for (int i = lane; i < m * B; i += kWave) hist_l[i] = 0;
    for (int j = lane; j < m; j += kWave) K[j] = A.vars[(int64_t)j * A.n + A.sites[s]];
    wave_sync();
    uint32_t vv[VPT];
    bool ok[VPT];
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int q = lane + i * kWave;
      ok[i] = q < nt;
      vv[i] = ok[i] ? A.perm[start + q] : 0u;
    }
#pragma unroll 2
    for (int j = 0; j < m; ++j) {
      const float kj = K[j];
      const float *col = A.vars + (int64_t)j * A.n;
      float x[VPT];
#pragma unroll
      for (int i = 0; i < VPT; ++i) x[i] = ok[i] ? col[vv[i]] : 0.0f;
      uint32_t kmn = 0xFFFFFFFFu, kmx = 0u;
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        if (!ok[i]) continue;
        dv[j * ld + lane + i * kWave] = x[i] - kj;
        const uint32_t kk = f2key(x[i]);
        kmn = min(kmn, kk);
        kmx = max(kmx, kk);
      }
      kmn = wave_min_u32(kmn);
      kmx = wave_max_u32(kmx);
      if (lane == 0) {
        kmin_l[j] = kmn;
        kmax_l[j] = kmx;
      }
      if (B > 0) {
        const float *e = edg + j * (B + 1);
        const float e0 = e[0], sc = (float)B / (e[B] - e0);
#pragma unroll
        for (int i = 0; i < VPT; ++i) {
          if (i * kWave >= nt) break;
          if (ok[i]) atomicAdd(&hist_l[j * B + hist_bin(x[i], e, B, e0, sc)], 1u);
        }
      }
    }
    wave_sync();
    float hi[R], lo[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      hi[q] = lo[q] = 0.0f;
      const int u = R == 1 ? lane % U : lane + q * kWave;
      const bool worker = R == 1 ? lane < G * U : u < U;
      if (!worker) continue;
      // Σd_j as d_j times ones through the product path (see k_agg_cell)
      const float *dj, *dk;
      if (u < m) {
        dj = dv + u * ld;
        dk = ones;
      } else {
        const int p = u - m;
        dj = dv + A.pairs.j[p] * ld;
        dk = dv + A.pairs.k[p] * ld;
      }
      for (int v = grp; v < nt; v += G) {
        const float a = dj[v], b = dk[v];
        const float pr = a * b;
        const float pe = __builtin_fmaf(a, b, -pr);
        acc(hi[q], lo[q], pr, pe);
      }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int u = R == 1 ? lane % U : lane + q * kWave;
      const bool worker = R == 1 ? lane < G * U : u < U;
      if (worker) {
        ph[grp * U + u] = hi[q];
        pl[grp * U + u] = lo[q];
      }
    }
    wave_sync();
    for (int u = lane; u < U; u += kWave) {
      float H = 0.0f, Lo = 0.0f;
      for (int gg = 0; gg < G; ++gg) {
        acc(H, Lo, ph[gg * U + u], 0.0f);
        Lo += pl[gg * U + u];
      }
      A.part_hi[(int64_t)item * U + u] = H;
      A.part_lo[(int64_t)item * U + u] = Lo;
    }
    if (A.hist) {
      uint32_t *dst = A.hist + (int64_t)s * m * B;
      for (int i = lane; i < m * B; i += kWave)
        if (hist_l[i]) atomicAdd(&dst[i], hist_l[i]);
    }
    for (int j = lane; j < m; j += kWave) {
      if (kmin_l[j] != 0xFFFFFFFFu) atomicMin(&A.kmin[(int64_t)s * m + j], kmin_l[j]);
      if (kmax_l[j] != 0u) atomicMax(&A.kmax[(int64_t)s * m + j], kmax_l[j]);
    }
    wave_sync();
  }
}

// 4. per-cell finalize: combine item partials (item order), form the float32
// statistics and the float64 merge inputs.
struct FinArgs {
  uint32_t S;
  int m, U, P;  // P = number of pair units (all pairs, or the diagonal only)
  Pairs pairs;
  const uint32_t *sites;
  const float *vars;
  int64_t n;
  const unsigned long long *cnt;
  const uint32_t *rank;      // site -> cell rank
  const uint32_t *item_off;  // by rank
  const float *part_hi, *part_lo;
  const uint32_t *kmin, *kmax;
  // outputs
  uint64_t *out_n;
  float *mean32, *m2_32, *vmin, *vmax, *cov32;  // cov32 [S][m(m+1)/2] (only with cov)
  int with_cov;
  double *mean64;  // [S][m]
  double *c64;     // [S][P]
  // exact merges into the components
  int B;
  const uint32_t *hist;           // cell histograms [S][m][B] or null
  const uint32_t *site_comp;
  uint32_t n_comp;
  unsigned long long *cnt_c;
  uint32_t *kmin_c, *kmax_c, *hist_c;
};

__global__ __launch_bounds__(kAggThreads) void k_agg_finalize(FinArgs A) {
  extern __shared__ uint8_t smem[];
  float *th = reinterpret_cast<float *>(smem);  // [U]
  float *tl = th + A.U;                         // [U]
  float *K = tl + A.U;                          // [m]
  const int t = threadIdx.x;
  const int m = A.m;
  for (uint32_t s = blockIdx.x; s < A.S; s += gridDim.x) {
    const uint64_t n = A.cnt[s];
    const uint32_t i0 = A.item_off[A.rank[s]], i1 = A.item_off[A.rank[s] + 1];
    for (int u = t; u < A.U; u += kAggThreads) {
      float H = 0.0f, Lo = 0.0f;
      for (uint32_t it = i0; it < i1; ++it) {
        acc(H, Lo, A.part_hi[(int64_t)it * A.U + u], 0.0f);
        Lo += A.part_lo[(int64_t)it * A.U + u];
      }
      th[u] = H;
      tl[u] = Lo;
    }
    if (t < m) K[t] = n ? A.vars[(int64_t)t * A.n + A.sites[s]] : 0.0f;
    __syncthreads();
    if (t == 0) A.out_n[s] = n;
    const uint32_t c = A.site_comp[s];
    if (n && c < A.n_comp) {
      if (t == 0) atomicAdd(&A.cnt_c[c], (unsigned long long)n);
      for (int j = t; j < m; j += kAggThreads) {
        atomicMin(&A.kmin_c[(int64_t)c * m + j], A.kmin[(int64_t)s * m + j]);
        atomicMax(&A.kmax_c[(int64_t)c * m + j], A.kmax[(int64_t)s * m + j]);
      }
      if (A.hist)
        for (int i = t; i < m * A.B; i += kAggThreads) {
          uint32_t h = A.hist[(int64_t)s * m * A.B + i];
          if (h) atomicAdd(&A.hist_c[(int64_t)c * m * A.B + i], h);
        }
    }
    const double dn = (double)n;
    for (int j = t; j < m; j += kAggThreads) {
      float mean = 0.0f;
      double mean64 = 0.0;
      if (n) {
        // the compensated pair (th, tl) is exact in float64; the float32
        // output is the float64 result rounded once
        mean64 = (double)K[j] + ((double)th[j] + (double)tl[j]) / dn;
        mean = (float)mean64;
      }
      A.mean32[(int64_t)s * m + j] = mean;
      A.mean64[(int64_t)s * m + j] = mean64;
      A.vmin[(int64_t)s * m + j] = n ? key2f(A.kmin[(int64_t)s * m + j]) : __builtin_inff();
      A.vmax[(int64_t)s * m + j] = n ? key2f(A.kmax[(int64_t)s * m + j]) : -__builtin_inff();
    }
    for (int p = t; p < A.P; p += kAggThreads) {
      const int j = A.pairs.j[p], k = A.pairs.k[p];
      float c32 = 0.0f;
      double c64 = 0.0;
      if (n) {
        // C = S_jk - S_j S_k / n cancels when the site's value is far from the
        // cell mean, so it is formed in float64 from the exact pairs and the
        // float32 output is that result rounded once
        const int uq = m + p;
        double dj = (double)th[j] + (double)tl[j], dk = (double)th[k] + (double)tl[k];
        c64 = ((double)th[uq] + (double)tl[uq]) - dj * dk / dn;
        if (j == k && c64 < 0.0) c64 = 0.0;
        c32 = (float)c64;
      }
      A.c64[(int64_t)s * A.P + p] = c64;
      if (j == k) A.m2_32[(int64_t)s * m + j] = c32;
      if (A.with_cov) A.cov32[(int64_t)s * A.P + p] = c32;
    }
    __syncthreads();
  }
}

// 5a. exact band statistics from the components: one workgroup per run of 256
// components in band order; each lane owns columns (count, minima, maxima,
// histogram bins) and flushes one atomic per column whenever the band changes.
struct BandIntArgs {
  uint32_t n_comp;
  int m, B;
  const uint32_t *order;  // components sorted by band
  const uint8_t *comp_band;
  const unsigned long long *cnt_c;
  const uint32_t *kmin_c, *kmax_c, *hist_c;
  unsigned long long *cnt_b;
  uint32_t *kmin_b, *kmax_b, *hist_b;
};

__global__ __launch_bounds__(256) void k_band_int(BandIntArgs A) {
  const int m = A.m, B = A.B;
  const int64_t cols = 1 + 2 * (int64_t)m + (int64_t)m * B;
  const uint32_t q0 = blockIdx.x * 256u;
  const uint32_t q1 = q0 + 256u < A.n_comp ? q0 + 256u : A.n_comp;
  const int nq = (int)(q1 - q0);
  // the run's components and their bands, staged once (the order -> band
  // chain of loads would otherwise repeat for every column)
  __shared__ uint32_t cs[256];
  __shared__ int bs[256];
  if ((int)threadIdx.x < nq) {
    const uint32_t c = A.order[q0 + threadIdx.x];
    cs[threadIdx.x] = c;
    bs[threadIdx.x] = A.comp_band[c];
  }
  __syncthreads();
  constexpr int kAhead = 8;  // loads issued together per column
  for (int64_t col = threadIdx.x; col < cols; col += 256) {
    const int kind = col == 0 ? 0 : col <= m ? 1 : col <= 2 * m ? 2 : 3;
    const int64_t sub = kind == 1 ? col - 1 : kind == 2 ? col - 1 - m : col - 1 - 2 * m;
    uint64_t acc = kind == 1 ? 0xFFFFFFFFull : 0ull;
    int band = -1;
    auto flush = [&]() {
      if (band < 0) return;
      if (kind == 0) {
        if (acc) atomicAdd(&A.cnt_b[band], (unsigned long long)acc);
      } else if (kind == 1) {
        if (acc != 0xFFFFFFFFull) atomicMin(&A.kmin_b[(int64_t)band * m + sub], (uint32_t)acc);
      } else if (kind == 2) {
        if (acc) atomicMax(&A.kmax_b[(int64_t)band * m + sub], (uint32_t)acc);
      } else {
        if (acc) atomicAdd(&A.hist_b[(int64_t)band * m * B + sub], (uint32_t)acc);
      }
    };
    for (int q = 0; q < nq; q += kAhead) {
      uint64_t v[kAhead];
#pragma unroll
      for (int k = 0; k < kAhead; ++k) {
        v[k] = 0;
        if (q + k >= nq) continue;
        const uint32_t c = cs[q + k];
        v[k] = kind == 0 ? (uint64_t)A.cnt_c[c]
             : kind == 1 ? (uint64_t)A.kmin_c[(int64_t)c * m + sub]
             : kind == 2 ? (uint64_t)A.kmax_c[(int64_t)c * m + sub]
                         : (uint64_t)A.hist_c[(int64_t)c * m * B + sub];
      }
#pragma unroll
      for (int k = 0; k < kAhead; ++k) {
        if (q + k >= nq) break;
        const int bc = bs[q + k];
        if (bc != band) {
          flush();
          band = bc;
          acc = kind == 1 ? 0xFFFFFFFFull : 0ull;
        }
        if (kind == 0 || kind == 3)
          acc += v[k];
        else if (kind == 1)
          acc = v[k] < acc ? v[k] : acc;
        else
          acc = v[k] > acc ? v[k] : acc;
      }
    }
    flush();
  }
}

__global__ void k_decode_minmax(const uint32_t *kmin, const uint32_t *kmax, const unsigned long long *cnt, int64_t units,
                                int m, float *vmin, float *vmax, uint64_t *out_n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= units * m) return;
  int64_t u = i / m;
  bool any = cnt[u] != 0;
  vmin[i] = any ? key2f(kmin[i]) : __builtin_inff();
  vmax[i] = any ? key2f(kmax[i]) : -__builtin_inff();
  if (i % m == 0) out_n[u] = cnt[u];
}

// 5b. Chan pairwise merge in float64.  Members of group g are
// order[off[g] .. off[g+1]) in that order.  Groups of at most kSmallGroup
// members: one thread per (group, pair unit) merges them one after another.
// Larger groups: one workgroup per (group, pair unit); lane t merges its
// contiguous share of the members in order, then the 256 lane states merge
// pairwise in a fixed tree (t with t + 128, ..., t with t + 1).
constexpr uint32_t kSmallGroup = 32;

struct MergeArgs {
  uint32_t n_groups;
  int m, P;
  Pairs pairs;
  const uint32_t *order;
  const uint32_t *off;
  const unsigned long long *in_cnt;
  const double *in_mean;           // [members][m]
  const double *in_c;              // [members][P]
  double *out_mean;                // [groups][m]
  double *out_m2;                  // [groups][m]
  double *out_c;                   // [groups][P] (internal, always)
  double *out_cov;                 // [groups][P] user output, or null
  int with_cov;
  const uint32_t *big;             // groups larger than kSmallGroup
  const uint32_t *big_cnt;
};

struct ChanState {
  double n, mj, mk, c;
};

__device__ __forceinline__ void chan_add(ChanState &a, double ni, double aj, double ak, double ci) {
  if (ni == 0.0) return;
  if (a.n == 0.0) {
    a = ChanState{ni, aj, ak, ci};
    return;
  }
  const double nn = a.n + ni;
  const double dj = aj - a.mj, dk = ak - a.mk;
  a.c = a.c + ci + dj * dk * (a.n * ni / nn);
  a.mj = a.mj + dj * (ni / nn);
  a.mk = a.mk + dk * (ni / nn);
  a.n = nn;
}

__device__ __forceinline__ void chan_write(const MergeArgs &A, uint32_t gidx, int p, const ChanState &st) {
  const int j = A.pairs.j[p], k = A.pairs.k[p];
  A.out_c[(int64_t)gidx * A.P + p] = st.c;
  if (j == k) {
    A.out_mean[(int64_t)gidx * A.m + j] = st.mj;
    A.out_m2[(int64_t)gidx * A.m + j] = st.c;
  }
  if (A.with_cov) A.out_cov[(int64_t)gidx * A.P + p] = st.c;
}

__global__ void k_chan_small(MergeArgs A) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)A.n_groups * A.P) return;
  const uint32_t gidx = (uint32_t)(i / A.P);
  const int p = (int)(i % A.P);
  const uint32_t q0 = A.off[gidx], q1 = A.off[gidx + 1];
  if (q1 - q0 > kSmallGroup) return;
  const int j = A.pairs.j[p], k = A.pairs.k[p];
  ChanState st{0.0, 0.0, 0.0, 0.0};
  for (uint32_t q = q0; q < q1; ++q) {
    const uint32_t mem = A.order[q];
    chan_add(st, (double)A.in_cnt[mem], A.in_mean[(int64_t)mem * A.m + j], A.in_mean[(int64_t)mem * A.m + k],
             A.in_c[(int64_t)mem * A.P + p]);
  }
  chan_write(A, gidx, p, st);
}

__global__ void k_chan_list_big(const uint32_t *off, uint32_t n_groups, uint32_t *big, uint32_t *big_cnt) {
  uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n_groups && off[g + 1] - off[g] > kSmallGroup) big[atomicAdd(big_cnt, 1u)] = g;
}

__global__ __launch_bounds__(256) void k_chan_big(MergeArgs A) {
  __shared__ double sn[256], sj[256], sk[256], sc[256];
  const int t = threadIdx.x;
  const int64_t work = (int64_t)(*A.big_cnt) * A.P;
  for (int64_t w = blockIdx.x; w < work; w += gridDim.x) {
    const uint32_t gidx = A.big[w / A.P];
    const int p = (int)(w % A.P);
    const int j = A.pairs.j[p], k = A.pairs.k[p];
    const uint32_t q0 = A.off[gidx], q1 = A.off[gidx + 1];
    const uint32_t len = q1 - q0, share = (len + 255) / 256;
    const uint32_t a0 = q0 + t * share;
    const uint32_t a1 = a0 + share < q1 ? a0 + share : q1;
    ChanState st{0.0, 0.0, 0.0, 0.0};
    for (uint32_t q = a0; q < a1; ++q) {
      const uint32_t mem = A.order[q];
      chan_add(st, (double)A.in_cnt[mem], A.in_mean[(int64_t)mem * A.m + j], A.in_mean[(int64_t)mem * A.m + k],
               A.in_c[(int64_t)mem * A.P + p]);
    }
    sn[t] = st.n;
    sj[t] = st.mj;
    sk[t] = st.mk;
    sc[t] = st.c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (t < o) {
        ChanState a{sn[t], sj[t], sk[t], sc[t]};
        chan_add(a, sn[t + o], sj[t + o], sk[t + o], sc[t + o]);
        sn[t] = a.n;
        sj[t] = a.mj;
        sk[t] = a.mk;
        sc[t] = a.c;
      }
      __syncthreads();
    }
    if (t == 0) chan_write(A, gidx, p, ChanState{sn[0], sj[0], sk[0], sc[0]});
    __syncthreads();
  }
}

// helpers for ordering components by band
__global__ void k_permute(const uint32_t *key, const uint32_t *val, const uint32_t *pos, uint32_t n, uint32_t *key_out,
                          uint32_t *val_out) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    key_out[pos[i]] = key[i];
    val_out[pos[i]] = val[i];
  }
}
__global__ void k_iota(uint32_t *p, uint32_t n) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

struct AggWork {
  LayoutWork lay;
  uint32_t *perm;  // [N]
  unsigned long long *cnt_c, *cnt_b;
  uint32_t *items, *item_off;
  float *part_hi, *part_lo;
  uint32_t *kmin, *kmax, *kmin_c, *kmax_c, *kmin_b, *kmax_b;
  double *mean64, *c64, *mean64_c, *c64_c, *m2tmp_c, *mean64_b, *c64_b, *m2tmp_b;
  uint32_t *key_b, *val_b, *pos, *corder, *bucket;
  uint32_t *item_rank, *small_list, *big_list, *big, *big_cnt;
  void *scratch;
  size_t scratch_bytes;
  int64_t item_cap;
};

// Items: one per started kItemVoxels of every cell.
int64_t item_capacity(const Geom &g, uint32_t S) { return (int64_t)S + g.n / kItemVoxels + 1; }

template <class A>
void agg_layout(A &a, const Geom &g, uint32_t S, uint32_t n_comp, int32_t n_bands, int m, int U, int P, AggWork *W) {
  size_t s1 = S ? S : 1, c1 = n_comp + 2, b1 = (size_t)n_bands + 1;
  int64_t ic = item_capacity(g, S);
  layout_take(a, g, S, n_comp, W ? &W->lay : nullptr);
  auto perm = a.template take<uint32_t>(g.n);
  auto cnt_c = a.template take<unsigned long long>(c1);
  auto cnt_b = a.template take<unsigned long long>(b1);
  auto items = a.template take<uint32_t>(s1);
  auto ioff = a.template take<uint32_t>(s1 + 1);
  auto ph = a.template take<float>(ic * U);
  auto pl = a.template take<float>(ic * U);
  auto kmin = a.template take<uint32_t>(s1 * m);
  auto kmax = a.template take<uint32_t>(s1 * m);
  auto kminc = a.template take<uint32_t>(c1 * m);
  auto kmaxc = a.template take<uint32_t>(c1 * m);
  auto kminb = a.template take<uint32_t>(b1 * m);
  auto kmaxb = a.template take<uint32_t>(b1 * m);
  auto mean64 = a.template take<double>(s1 * m);
  auto c64 = a.template take<double>(s1 * P);
  auto mean64c = a.template take<double>(c1 * m);
  auto c64c = a.template take<double>(c1 * P);
  auto m2c = a.template take<double>(c1 * m);
  auto mean64b = a.template take<double>(b1 * m);
  auto c64b = a.template take<double>(b1 * P);
  auto m2b = a.template take<double>(b1 * m);
  auto kb = a.template take<uint32_t>(c1);
  auto vb = a.template take<uint32_t>(c1);
  auto pos = a.template take<uint32_t>(c1);
  auto corder = a.template take<uint32_t>(c1);
  auto bucket = a.template take<uint32_t>(257);
  auto irank = a.template take<uint32_t>(ic);
  auto slist = a.template take<uint32_t>(ic);
  auto blist = a.template take<uint32_t>(ic);
  auto big = a.template take<uint32_t>(c1 > b1 ? c1 : b1);
  auto bigc = a.template take<uint32_t>(4);
  if (W) {
    W->perm = perm;
    W->cnt_c = cnt_c;
    W->cnt_b = cnt_b;
    W->items = items;
    W->item_off = ioff;
    W->part_hi = ph;
    W->part_lo = pl;
    W->kmin = kmin;
    W->kmax = kmax;
    W->kmin_c = kminc;
    W->kmax_c = kmaxc;
    W->kmin_b = kminb;
    W->kmax_b = kmaxb;
    W->mean64 = mean64;
    W->c64 = c64;
    W->mean64_c = mean64c;
    W->c64_c = c64c;
    W->m2tmp_c = m2c;
    W->mean64_b = mean64b;
    W->c64_b = c64b;
    W->m2tmp_b = m2b;
    W->key_b = kb;
    W->val_b = vb;
    W->pos = pos;
    W->corder = corder;
    W->bucket = bucket;
    W->item_rank = irank;
    W->small_list = slist;
    W->big_list = blist;
    W->big = big;
    W->big_cnt = bigc;
    W->item_cap = ic;
  }
}

struct SizerT : Sizer {
  template <class T>
  T *take(size_t c) {
    Sizer::take<T>(c);
    return nullptr;
  }
};

void units_for(int m, bool cov, int &P, int &U, Pairs &pairs) {
  P = 0;
  for (int j = 0; j < m; ++j)
    for (int k = j; k < m; ++k)
      if (cov || j == k) {
        pairs.j[P] = (uint8_t)j;
        pairs.k[P] = (uint8_t)k;
        ++P;
      }
  U = m + P;
}

size_t scratch_need(const Geom &g, uint32_t S, uint32_t n_comp) {
  size_t a = ScanU32::workspace((int64_t)S + 1);
  size_t b = StableSort8::workspace((int64_t)n_comp + 2);
  size_t c = ScanU32::workspace((int64_t)n_comp + 2);
  size_t d = layout_scratch(g, S, n_comp);
  size_t r = a > b ? a : b;
  r = r > c ? r : c;
  return (r > d ? r : d) + 256;
}

}  // namespace

}  // namespace lsrvt

using namespace lsrvt;

extern "C" size_t lsrvt_aggregate_workspace(lsrvt_dims dims, uint32_t n_sites, uint32_t n_comp, int32_t n_bands,
                                            int32_t n_vars, int32_t n_bins, uint32_t flags) {
  (void)n_bins;
  Geom g;
  if (make_geom(dims, g)) return 0;
  if (n_vars < 1 || n_vars > kMaxVars || n_bands < 1 || n_bands > 255) return 0;
  int P, U;
  Pairs pairs;
  units_for(n_vars, (flags & LSRVT_STATS_COV) != 0, P, U, pairs);
  SizerT z;
  agg_layout(z, g, n_sites, n_comp, n_bands, n_vars, U, P, nullptr);
  return z.off + scratch_need(g, n_sites, n_comp);
}

extern "C" int32_t lsrvt_aggregate(const uint32_t *d_cell, lsrvt_dims dims, const uint32_t *d_sites,
                                   const uint32_t *d_site_comp, uint32_t n_sites, const uint8_t *d_comp_band,
                                   uint32_t n_comp, int32_t n_bands, const float *d_vars, int32_t n_vars,
                                   const float *d_edges, int32_t n_bins, uint32_t flags, const lsrvt_cell_stats *cell,
                                   const lsrvt_group_stats *comp, const lsrvt_group_stats *band, void *d_work,
                                   size_t work_bytes, void *stream) {
  Geom g;
  int32_t rc = make_geom(dims, g);
  if (rc) return rc;
  if (n_vars < 1 || n_vars > kMaxVars || n_bands < 1 || n_bands > 255) return LSRVT_EINVAL;
  if (!d_cell || !d_vars || !cell || !comp || !band) return LSRVT_EINVAL;
  if (n_sites && (!d_sites || !d_site_comp)) return LSRVT_EINVAL;
  if (n_comp && !d_comp_band) return LSRVT_EINVAL;
  const bool want_hist = (flags & LSRVT_STATS_HIST) != 0;
  const bool want_cov = (flags & LSRVT_STATS_COV) != 0;
  const int B = want_hist ? n_bins : 0;
  if (want_hist && (n_bins < 1 || !d_edges || (int64_t)n_vars * n_bins > kMaxHist)) return LSRVT_EINVAL;
  const lsrvt_cell_stats &cs = *cell;
  const lsrvt_group_stats *lv[2] = {comp, band};
  if (!cs.n || !cs.mean || !cs.m2 || !cs.vmin || !cs.vmax || (want_hist && !cs.hist) || (want_cov && !cs.cov))
    return LSRVT_EINVAL;
  for (const lsrvt_group_stats *q : lv)
    if (!q->n || !q->mean || !q->m2 || !q->vmin || !q->vmax || (want_hist && !q->hist) || (want_cov && !q->cov))
      return LSRVT_EINVAL;
  const size_t need = lsrvt_aggregate_workspace(dims, n_sites, n_comp, n_bands, n_vars, n_bins, flags);
  if ((rc = check_work(d_work, work_bytes, need))) return rc;
  int P, U;
  Pairs pairs;
  units_for(n_vars, want_cov, P, U, pairs);
  const int m = n_vars;
  Carve cv(d_work, work_bytes);
  AggWork W;
  agg_layout(cv, g, n_sites, n_comp, n_bands, m, U, P, &W);
  if (!cv.ok) return LSRVT_EWORKSPACE;
  W.scratch = cv.base + cv.off;
  W.scratch_bytes = cv.size - cv.off;
  hipStream_t s = as_stream(stream);
  const uint32_t S = n_sites;
  const uint32_t C = n_comp;
  const int64_t Pfull = (int64_t)m * (m + 1) / 2;

  // zero / identity initialisation
  if ((rc = fill<unsigned long long>(W.cnt_c, C + 2, 0ull, s))) return rc;
  if ((rc = fill<unsigned long long>(W.cnt_b, n_bands + 1, 0ull, s))) return rc;
  if ((rc = fill<uint32_t>(W.kmin, (int64_t)(S ? S : 1) * m, 0xFFFFFFFFu, s))) return rc;
  if ((rc = fill<uint32_t>(W.kmax, (int64_t)(S ? S : 1) * m, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(W.kmin_c, (int64_t)(C + 2) * m, 0xFFFFFFFFu, s))) return rc;
  if ((rc = fill<uint32_t>(W.kmax_c, (int64_t)(C + 2) * m, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(W.kmin_b, (int64_t)(n_bands + 1) * m, 0xFFFFFFFFu, s))) return rc;
  if ((rc = fill<uint32_t>(W.kmax_b, (int64_t)(n_bands + 1) * m, 0u, s))) return rc;
  if (want_hist) {
    if ((rc = fill<uint32_t>(cs.hist, (int64_t)S * m * B, 0u, s))) return rc;
    if ((rc = fill<uint32_t>(comp->hist, (int64_t)C * m * B, 0u, s))) return rc;
    if ((rc = fill<uint32_t>(band->hist, (int64_t)n_bands * m * B, 0u, s))) return rc;
  }

  // 1. sites in (component, id) order and the voxels of every cell as one range
  W.lay.scratch = W.scratch;
  W.lay.scratch_bytes = W.scratch_bytes;
  if ((rc = layout_sites(d_site_comp, S, C, W.lay, s))) return rc;
  if ((rc = layout_voxels(d_cell, g, S, W.lay, W.perm, s))) return rc;

  // 2. items
  uint32_t n_items = 0;
  if (S) {
    hipLaunchKernelGGL(k_agg_items, dim3((S + 255) / 256), dim3(256), 0, s, W.lay.cnt_rank, S, W.items);
    LSRVT_LAUNCHED();
    if ((rc = ScanU32::run(W.items, S, W.item_off, W.scratch, W.scratch_bytes, s))) return rc;
    {
      const int32_t rc_ = read_words(W.item_off + S, 1, &n_items, s);
      if (rc_) return rc_;
    }
    if ((int64_t)n_items > W.item_cap) return LSRVT_EDEVICE;  // cannot happen: the capacity is an upper bound
  }

  // 3. per-item sums: cells of at most kSmallCell voxels one wave each, larger cells one workgroup per item
  if (n_items) {
    CellArgs A;
    A.perm = W.perm;
    A.cell_off = W.lay.cell_off;
    A.order = W.lay.order;
    A.sites = d_sites;
    A.vars = d_vars;
    A.edges = d_edges;
    A.n = g.n;
    A.m = m;
    A.B = B;
    A.U = U;
    A.P = P;
    A.pairs = pairs;
    A.item_off = W.item_off;
    A.item_rank = W.item_rank;
    A.part_hi = W.part_hi;
    A.part_lo = W.part_lo;
    A.hist = want_hist ? cs.hist : nullptr;
    A.kmin = W.kmin;
    A.kmax = W.kmax;
    // wave path: U units over 64 lanes, LDS for four waves
    const int Rw = (U + kWave - 1) / kWave;
    const int Gw = Rw == 1 ? kWave / U : 1;
    const size_t lds_w =
        sizeof(float) * ((size_t)m * (B + 1) + kSmallCell + 1 + (kAggThreads / kWave) * wave_region_words(m, B, U, Gw));
    const bool small_ok = Rw <= 3 && lds_w <= 65536;
    if ((rc = fill<uint32_t>(W.big_cnt + 1, 2, 0u, s))) return rc;
    uint32_t *counts = W.big_cnt + 1;
    hipLaunchKernelGGL(k_item_cells, dim3((S + 255) / 256), dim3(256), 0, s, W.item_off, W.lay.cnt_rank, S,
                       small_ok ? 1 : 0, W.item_rank, W.small_list, W.big_list, counts);
    LSRVT_LAUNCHED();
    if (small_ok) {
      A.list = W.small_list;
      A.list_cnt = counts;
      A.G = Gw;
      A.tile = kSmallCell;
      const unsigned grid = (unsigned)std::min<uint64_t>(65535, (n_items + 3) / 4);
      if (Rw == 1)
        hipLaunchKernelGGL(k_agg_cell_wave<1>, dim3(grid), dim3(kAggThreads), lds_w, s, A);
      else if (Rw == 2)
        hipLaunchKernelGGL(k_agg_cell_wave<2>, dim3(grid), dim3(kAggThreads), lds_w, s, A);
      else
        hipLaunchKernelGGL(k_agg_cell_wave<3>, dim3(grid), dim3(kAggThreads), lds_w, s, A);
      LSRVT_LAUNCHED();
    }
    A.list = W.big_list;
    A.list_cnt = counts + 1;
    const int R = (U + kAggThreads - 1) / kAggThreads;
    // lane groups: 256 / U of them in 256 threads while units fill at most
    // half the workgroup, else two groups in up to 512 threads (all lanes but
    // the rounding to whole waves work)
    int NT = kAggThreads;
    if (R == 1) {
      A.G = 2 * U <= kAggThreads ? kAggThreads / U : 2;
      NT = std::max(kAggThreads, (A.G * U + kWave - 1) / kWave * kWave);
    } else {
      A.G = 1;
    }
    // the largest staging round (NT, 2 NT or 4 NT voxels) that keeps the
    // workgroup within 40 KiB of LDS, so four workgroups share a CU
    const size_t fixed = sizeof(float) * ((size_t)m * B + 3 * m + 2 * (size_t)A.G * U + (size_t)m * (B + 1) + m);
    size_t lds = 0;
    int vpt = kMaxVPT;
    for (; vpt >= 1; vpt /= 2) {
      A.tile = vpt * NT;
      lds = fixed + sizeof(float) * (size_t)(m + 1) * (A.tile + 4);
      if (lds <= 40960 || vpt == 1) break;
    }
    const int32_t tv = tuning(LSRVT_TUNE_STATS_TILE);  // a tuned round size, if it fits in 64 KiB
    if (tv) {
      const size_t l2 = fixed + sizeof(float) * (size_t)(m + 1) * ((size_t)tv * NT + 4);
      if (l2 <= 65536) {
        vpt = tv;
        A.tile = vpt * NT;
        lds = l2;
      }
    }
    if (lds > 65536 || R > 3 || NT > kAggMaxThreads) return LSRVT_EINVAL;
    const unsigned grid = n_items < 16384 ? n_items : 16384;
    auto launch = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, s, A); };
    if (R == 1)
      vpt == 4 ? launch(k_agg_cell<1, 4>) : vpt == 2 ? launch(k_agg_cell<1, 2>) : launch(k_agg_cell<1, 1>);
    else if (R == 2)
      vpt == 4 ? launch(k_agg_cell<2, 4>) : vpt == 2 ? launch(k_agg_cell<2, 2>) : launch(k_agg_cell<2, 1>);
    else
      vpt == 4 ? launch(k_agg_cell<3, 4>) : vpt == 2 ? launch(k_agg_cell<3, 2>) : launch(k_agg_cell<3, 1>);
    LSRVT_LAUNCHED();
  }

  // 4. per-cell finalize, plus exact merges of counts, extrema and histograms into components
  if (S) {
    FinArgs F;
    F.S = S;
    F.m = m;
    F.U = U;
    F.P = P;
    F.pairs = pairs;
    F.sites = d_sites;
    F.vars = d_vars;
    F.n = g.n;
    F.cnt = W.lay.cnt;
    F.rank = W.lay.rank;
    F.item_off = W.item_off;
    F.part_hi = W.part_hi;
    F.part_lo = W.part_lo;
    F.kmin = W.kmin;
    F.kmax = W.kmax;
    F.out_n = cs.n;
    F.mean32 = cs.mean;
    F.m2_32 = cs.m2;
    F.vmin = cs.vmin;
    F.vmax = cs.vmax;
    F.cov32 = cs.cov;
    F.with_cov = want_cov;
    F.mean64 = W.mean64;
    F.c64 = W.c64;
    F.B = B;
    F.hist = want_hist ? cs.hist : nullptr;
    F.site_comp = d_site_comp;
    F.n_comp = C;
    F.cnt_c = W.cnt_c;
    F.kmin_c = W.kmin_c;
    F.kmax_c = W.kmax_c;
    F.hist_c = want_hist ? comp->hist : nullptr;
    size_t lds = sizeof(float) * (2 * (size_t)U + m);
    hipLaunchKernelGGL(k_agg_finalize, dim3(S < 16384 ? S : 16384), dim3(kAggThreads), lds, s, F);
    LSRVT_LAUNCHED();
  }

  // 5a. components sorted by band (stable in id); exact band statistics
  if (C) {
    hipLaunchKernelGGL(k_iota, dim3((C + 255) / 256), dim3(256), 0, s, W.corder, C);
    LSRVT_LAUNCHED();
    if ((rc = StableSort8::run(d_comp_band, C, W.pos, W.bucket, W.scratch, W.scratch_bytes, s))) return rc;
    hipLaunchKernelGGL(k_permute, dim3((C + 255) / 256), dim3(256), 0, s, W.corder, W.corder, W.pos, C, W.key_b,
                       W.val_b);
    LSRVT_LAUNCHED();
    BandIntArgs BI;
    BI.n_comp = C;
    BI.m = m;
    BI.B = B;
    BI.order = W.val_b;
    BI.comp_band = d_comp_band;
    BI.cnt_c = W.cnt_c;
    BI.kmin_c = W.kmin_c;
    BI.kmax_c = W.kmax_c;
    BI.hist_c = want_hist ? comp->hist : nullptr;
    BI.cnt_b = W.cnt_b;
    BI.kmin_b = W.kmin_b;
    BI.kmax_b = W.kmax_b;
    BI.hist_b = want_hist ? band->hist : nullptr;
    hipLaunchKernelGGL(k_band_int, dim3((C + 255) / 256), dim3(256), 0, s, BI);
    LSRVT_LAUNCHED();
    hipLaunchKernelGGL(k_decode_minmax, dim3(grid_for((int64_t)C * m, 256, 1 << 30)), dim3(256), 0, s, W.kmin_c,
                       W.kmax_c, W.cnt_c, (int64_t)C, m, comp->vmin, comp->vmax, comp->n);
    LSRVT_LAUNCHED();
  } else {
    if ((rc = fill<uint32_t>(W.bucket, 257, 0u, s))) return rc;
  }
  hipLaunchKernelGGL(k_decode_minmax, dim3(grid_for((int64_t)n_bands * m, 256, 1 << 30)), dim3(256), 0, s, W.kmin_b,
                     W.kmax_b, W.cnt_b, (int64_t)n_bands, m, band->vmin, band->vmax, band->n);
  LSRVT_LAUNCHED();

  auto run_merge = [&](MergeArgs &M) -> int32_t {
    int32_t r;
    if ((r = fill<uint32_t>(W.big_cnt, 1, 0u, s))) return r;
    M.big = W.big;
    M.big_cnt = W.big_cnt;
    hipLaunchKernelGGL(k_chan_small, dim3(grid_for((int64_t)M.n_groups * M.P, 256, 1 << 30)), dim3(256), 0, s, M);
    hipLaunchKernelGGL(k_chan_list_big, dim3((M.n_groups + 255) / 256), dim3(256), 0, s, M.off, M.n_groups, W.big,
                       W.big_cnt);
    hipLaunchKernelGGL(k_chan_big, dim3(1024), dim3(256), 0, s, M);
    LSRVT_LAUNCHED();
    return LSRVT_OK;
  };

  // 5b. the cell -> component merge, cells of a component in site id order
  if (C) {
    if (S) {
      MergeArgs M;
      M.n_groups = C;
      M.m = m;
      M.P = P;
      M.pairs = pairs;
      M.order = W.lay.order;
      M.off = W.lay.coff;
      M.in_cnt = W.lay.cnt;
      M.in_mean = W.mean64;
      M.in_c = W.c64;
      M.out_mean = comp->mean;
      M.out_m2 = comp->m2;
      M.out_c = W.c64_c;
      M.out_cov = comp->cov;
      M.with_cov = want_cov;
      if ((rc = run_merge(M))) return rc;
      // keep float64 component means for the band merge
      LSRVT_HIP(hipMemcpyAsync(W.mean64_c, comp->mean, sizeof(double) * (size_t)C * m, hipMemcpyDeviceToDevice, s));
    } else {
      if ((rc = fill<double>(comp->mean, (int64_t)C * m, 0.0, s))) return rc;
      if ((rc = fill<double>(comp->m2, (int64_t)C * m, 0.0, s))) return rc;
      if (want_cov && (rc = fill<double>(comp->cov, (int64_t)C * Pfull, 0.0, s))) return rc;
      if ((rc = fill<double>(W.mean64_c, (int64_t)C * m, 0.0, s))) return rc;
      if ((rc = fill<double>(W.c64_c, (int64_t)C * P, 0.0, s))) return rc;
    }
  }

  // 5c. component -> band merge, components of a band in id order
  {
    MergeArgs M;
    M.n_groups = (uint32_t)n_bands;
    M.m = m;
    M.P = P;
    M.pairs = pairs;
    M.order = W.val_b;
    M.off = W.bucket;
    M.in_cnt = W.cnt_c;
    M.in_mean = W.mean64_c;
    M.in_c = W.c64_c;
    M.out_mean = band->mean;
    M.out_m2 = band->m2;
    M.out_c = W.c64_b;
    M.out_cov = band->cov;
    M.with_cov = want_cov;
    if ((rc = run_merge(M))) return rc;
  }
  return LSRVT_OK;
}
