// Stratified initial sites (Sec. 3.2.1, Eq. 3 and Eq. 4).
//
// Voxel mass m(v) = lut[w(v)] (m = w without a table, 1 without weights).
// A component C gets n_c = max(ceil(m(C) N / (rho M)), 1) sites, M the total
// mass and rho the voxels per site (Eq. 3 with the density as one site per
// rho voxels of average mass).  The volume is cut into cubes of edge B; the
// (component, block) pairs of C share its n_c sites by floor shares
// floor(n_c m(b) / m(C)) plus one each for the largest remainders
// n_c m(b) mod m(C), ties to the lower block index (Eq. 4, "most
// under-represented blocks").  Inside a pair, the n_b sites are placed by
// systematic sampling proportional to mass over the pair's voxels in
// linear-index order: with o in [0, m(b)) the j-th point is
// p_j = floor((o + j m(b)) / n_b) and the site is the voxel whose cumulative
// mass interval holds p_j.  o comes from Philox4x32-10 (Salmon et al., SC
// 2011) keyed by the seed, counter (block, component, 0, 0).  A component
// of zero mass gets one site, its first voxel (smallest linear index).  Sites are numbered by
// (component, block, j).  Every decision is taken in exact integer
// arithmetic, so the result does not depend on scheduling.
//
// Steps: per block, the distinct components and their masses (LDS hash);
// a scan gives the pairs block-major; a stable radix sort by component puts
// them in (component, block) order; one wave per component apportions its
// sites (the r-th largest remainder is found by bisection on its value);
// a scan numbers the sites; per block, each pair with sites runs a prefix
// sum of its mass over the block's voxels and places its points.
#include <algorithm>

#include "common.h"

namespace lsrvt {
namespace {

constexpr int kSeedThreads = 256;
constexpr int kMaxBlockEdge = 16;
constexpr int kBlockCap = kMaxBlockEdge * kMaxBlockEdge * kMaxBlockEdge;  // voxels (and components) per block

struct SeedGeom {
  Geom g;
  int32_t B;
  int32_t nbx, nby, nbz;
  int64_t nblocks;
};

SeedGeom seed_geom(const Geom &g, int32_t B) {
  SeedGeom G;
  G.g = g;
  G.B = B;
  G.nbx = (g.nx + B - 1) / B;
  G.nby = (g.ny + B - 1) / B;
  G.nbz = (g.nz + B - 1) / B;
  G.nblocks = (int64_t)G.nbx * G.nby * G.nbz;
  return G;
}

struct MassIn {
  const uint16_t *w;    // weights or null (mass 1)
  const uint32_t *lut;  // mass of every weight value or null (mass = weight)
};

__device__ __forceinline__ uint32_t voxel_mass(const MassIn &mi, int64_t v) {
  if (!mi.w) return 1u;
  const uint32_t x = mi.w[v];
  return mi.lut ? mi.lut[x] : x;
}

// Voxel k (x fastest) of block b as a linear index; -1 outside the volume.
// Within a block k increases with the linear index.
__device__ __forceinline__ int64_t block_voxel(const SeedGeom &G, int64_t b, int k) {
  const int bx = (int)(b % G.nbx), by = (int)((b / G.nbx) % G.nby), bz = (int)(b / ((int64_t)G.nbx * G.nby));
  const int x = bx * G.B + k % G.B, y = by * G.B + (k / G.B) % G.B, z = bz * G.B + k / (G.B * G.B);
  if (x >= G.g.nx || y >= G.g.ny || z >= G.g.nz) return -1;
  return x + (int64_t)G.g.nx * (y + (int64_t)G.g.ny * z);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (published multipliers and key increments)
struct U4 {
  uint32_t v[4];
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c.v[0], hi0 = __umulhi(0xD2511F53u, c.v[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c.v[2], hi1 = __umulhi(0xCD9E8D57u, c.v[2]);
    U4 o;
    o.v[0] = hi1 ^ c.v[1] ^ k0;
    o.v[1] = lo1;
    o.v[2] = hi0 ^ c.v[3] ^ k1;
    o.v[3] = lo0;
    c = o;
  }
  return c;
}

// ---------------------------------------------------------------------------
// exact 128-bit helpers
typedef unsigned __int128 u128;

__device__ __forceinline__ double u128_to_double(u128 a) {
  return (double)(uint64_t)(a >> 64) * 18446744073709551616.0 + (double)(uint64_t)a;
}

// floor(num / den) for a quotient below 2^32 (the estimate in double is then
// within one of it; the loops correct it exactly).  *err is set if the
// quotient is out of range.
__device__ __forceinline__ uint64_t div_small(u128 num, u128 den, uint32_t *err) {
  if (den == 0) {
    atomicOr(err, 2u);
    return 0;
  }
  double e = u128_to_double(num) / u128_to_double(den);
  if (!(e < 4294967296.0 * 2.0)) {
    atomicOr(err, 2u);
    return 0;
  }
  uint64_t q = (uint64_t)e;
  for (int i = 0; i < 4 && (u128)q * den > num; ++i) --q;
  for (int i = 0; i < 4 && (u128)(q + 1) * den <= num; ++i) ++q;
  if ((u128)q * den > num || (u128)(q + 1) * den <= num) atomicOr(err, 2u);
  return q;
}

// ---------------------------------------------------------------------------
// per block: distinct components (pass 0 counts them and sums the block's
// mass; pass 1 writes the pairs: component, block, mass)
template <int Pass>
__global__ __launch_bounds__(kSeedThreads) void k_seed_blocks(const uint32_t *__restrict__ comp, SeedGeom G,
                                                              uint32_t n_comp, MassIn mi, uint32_t *pcnt,
                                                              unsigned long long *bmass, const uint32_t *poff,
                                                              uint32_t *pair_comp, uint32_t *pair_block,
                                                              unsigned long long *pair_mass, uint32_t *err) {
  __shared__ uint32_t key[kBlockCap];
  __shared__ unsigned long long msum[Pass ? kBlockCap : 1];
  __shared__ uint32_t wsum[kSeedThreads / kWave];
  __shared__ unsigned long long red[Pass ? 1 : kSeedThreads];
  const int t = threadIdx.x;
  const int nv = G.B * G.B * G.B;
  for (int64_t b = blockIdx.x; b < G.nblocks; b += gridDim.x) {
    for (int i = t; i < kBlockCap; i += kSeedThreads) {
      key[i] = kNone;
      if (Pass) msum[i] = 0ull;
    }
    __syncthreads();
    unsigned long long mine = 0;
    for (int k = t; k < nv; k += kSeedThreads) {
      const int64_t v = block_voxel(G, b, k);
      if (v < 0) continue;
      const uint32_t c = comp[v];
      if (c >= n_comp) {
        atomicOr(err, 1u);
        continue;
      }
      const uint32_t m = voxel_mass(mi, v);
      mine += m;
      const int sl = lds_slot<kBlockCap>(key, c);  // a block holds at most kBlockCap components
      if (Pass && sl >= 0) atomicAdd(&msum[sl], (unsigned long long)m);
    }
    __syncthreads();
    // slots in use: count (pass 0) or compact in slot order (pass 1)
    constexpr int kPer = kBlockCap / kSeedThreads;
    uint32_t cnt = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) cnt += key[t * kPer + j] != kNone;
    const int lane = lane_id(), wid = t / kWave;
    uint32_t inc = cnt;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t x = __shfl_up(inc, o, kWave);
      if (lane >= o) inc += x;
    }
    if (lane == kWave - 1) wsum[wid] = inc;
    if (Pass == 0) red[t] = mine;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int q = 0; q < kSeedThreads / kWave; ++q) {
      if (q < wid) before += wsum[q];
      total += wsum[q];
    }
    if (Pass == 0) {
      for (int s = kSeedThreads / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
      }
      if (t == 0) {
        pcnt[b] = total;
        bmass[b] = red[0];
      }
    } else {
      uint32_t pos = poff[b] + before + inc - cnt;
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int sl = t * kPer + j;
        if (key[sl] != kNone) {
          pair_comp[pos] = key[sl];
          pair_block[pos] = (uint32_t)b;
          pair_mass[pos] = msum[sl];
          ++pos;
        }
      }
    }
    __syncthreads();
  }
}

// Total mass: one workgroup over the per-block sums (fixed order).
__global__ __launch_bounds__(kSeedThreads) void k_seed_total(const unsigned long long *bmass, int64_t nb,
                                                             unsigned long long *total) {
  __shared__ unsigned long long red[kSeedThreads];
  unsigned long long s = 0;
  for (int64_t i = threadIdx.x; i < nb; i += kSeedThreads) s += bmass[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = kSeedThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = red[0];
}

__global__ void k_seed_iota(uint32_t *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (uint32_t)i;
}

__global__ void k_seed_digit(const uint32_t *val, int64_t n, const uint32_t *pair_comp, int shift, uint8_t *digit) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) digit[i] = (uint8_t)(pair_comp[val[i]] >> shift);
}

__global__ void k_seed_scatter(const uint32_t *src, const uint32_t *pos, int64_t n, uint32_t *dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[pos[i]] = src[i];
}

// sorted views of the pairs and the segment of every component
__global__ void k_seed_sorted(const uint32_t *idx, int64_t P, const uint32_t *pair_comp,
                              const unsigned long long *pair_mass, uint32_t *scomp, unsigned long long *smass,
                              uint32_t *cbeg, uint32_t *cend) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const uint32_t c = pair_comp[idx[i]];
  scomp[i] = c;
  smass[i] = pair_mass[idx[i]];
  if (i == 0 || pair_comp[idx[i - 1]] != c) cbeg[c] = (uint32_t)i;
  if (i == P - 1 || pair_comp[idx[i + 1]] != c) cend[c] = (uint32_t)(i + 1);
}

// One wave per component: n_c and the share of each of its pairs (sorted
// order, blocks ascending), written to snb.
__global__ __launch_bounds__(kSeedThreads) void k_seed_apportion(uint32_t n_comp, const uint32_t *cbeg,
                                                                 const uint32_t *cend, const uint32_t *idx,
                                                                 const unsigned long long *smass,
                                                                 const unsigned long long *total, int64_t N,
                                                                 uint32_t rho, unsigned long long *srem,
                                                                 uint32_t *snb, uint32_t *err) {
  const int lane = lane_id();
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const u128 den = (u128)rho * (u128)(*total);
  for (int64_t c = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; c < n_comp; c += waves) {
    const uint32_t b0 = cbeg[c], b1 = cend[c];
    if (b1 <= b0) continue;
    unsigned long long mc = 0;
    for (uint32_t i = b0 + lane; i < b1; i += kWave) mc += smass[i];
    mc = wave_sum_u64(mc);
    if (mc == 0) {
      // zero mass: one site (the component's first voxel), numbered with its first pair
      for (uint32_t i = b0 + lane; i < b1; i += kWave) snb[i] = i == b0 ? 1u : 0u;
      continue;
    }
    // Eq. 3: n_c = max(ceil(m(C) N / (rho M)), 1)
    const u128 num = (u128)mc * (u128)(uint64_t)N;
    uint64_t nc = div_small(num, den, err);
    if ((u128)nc * den < num) ++nc;
    if (nc == 0) nc = 1;
    // floor shares and remainders
    uint64_t given = 0;
    for (uint32_t i = b0 + lane; i < b1; i += kWave) {
      const u128 q = (u128)nc * (u128)smass[i];
      const uint64_t base = div_small(q, (u128)mc, err);
      srem[i] = (unsigned long long)(q - (u128)base * mc);
      snb[i] = (uint32_t)base;
      given += base;
    }
    given = wave_sum_u64(given);
    const uint64_t r = nc - given;
    if (r == 0) continue;
    // the r-th largest remainder v: the largest v with #(rem >= v) >= r
    unsigned long long lo = 0, hi = mc;
    while (hi - lo > 1) {
      const unsigned long long mid = lo + (hi - lo) / 2;
      uint64_t k = 0;
      for (uint32_t i0 = b0; i0 < b1; i0 += kWave) {
        const uint32_t i = i0 + lane;
        k += (uint64_t)__popcll(__ballot(i < b1 && srem[i] >= mid));
      }
      if (k >= r)
        lo = mid;
      else
        hi = mid;
    }
    // remainders above v all get one more; those equal to v in block order
    uint64_t above = 0;
    for (uint32_t i0 = b0; i0 < b1; i0 += kWave) {
      const uint32_t i = i0 + lane;
      above += (uint64_t)__popcll(__ballot(i < b1 && srem[i] > lo));
    }
    uint64_t ties = r - above;
    for (uint32_t i0 = b0; i0 < b1; i0 += kWave) {
      const uint32_t i = i0 + lane;
      const bool gt = i < b1 && srem[i] > lo;
      const bool eq = i < b1 && srem[i] == lo;
      const uint64_t em = __ballot(eq);
      const uint64_t rank = (uint64_t)__popcll(em & lanemask_lt());
      if (gt || (eq && rank < ties)) snb[i] += 1u;
      const uint64_t used = (uint64_t)__popcll(em);
      ties = ties > used ? ties - used : 0;
    }
  }
}

// back to block-major pair order
__global__ void k_seed_unsort(const uint32_t *idx, int64_t P, const uint32_t *snb, const uint32_t *ssoff,
                              uint32_t *nb_pair, uint32_t *soff_pair) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  nb_pair[idx[i]] = snb[i];
  soff_pair[idx[i]] = ssoff[i];
}

// Per block, each pair with sites: prefix sums of the pair's mass over the
// block's voxels in linear order, then the systematic points.  The block's
// components and masses are read once into registers (thread t holds voxels
// 16 t .. 16 t + 15); per pair the prefix sums are a wave scan of the
// per-thread sums plus the four wave totals.
__global__ __launch_bounds__(kSeedThreads) void k_seed_place(const uint32_t *__restrict__ comp, SeedGeom G,
                                                             MassIn mi, const uint32_t *poff,
                                                             const uint32_t *pair_comp,
                                                             const unsigned long long *pair_mass,
                                                             const uint32_t *comp_first, const uint32_t *nb_pair,
                                                             const uint32_t *soff_pair, uint32_t key_lo,
                                                             uint32_t key_hi, uint32_t *sites, uint32_t cap) {
  __shared__ unsigned long long cum[kBlockCap];
  __shared__ unsigned long long wtot[kSeedThreads / kWave];
  const int t = threadIdx.x, lane = lane_id(), wid = t / kWave;
  const int nv = G.B * G.B * G.B;
  constexpr int kPer = kBlockCap / kSeedThreads;
  for (int64_t b = blockIdx.x; b < G.nblocks; b += gridDim.x) {
    const uint32_t k0 = poff[b], k1 = poff[b + 1];
    uint32_t any = 0;
    for (uint32_t k = k0; k < k1; ++k) any |= nb_pair[k];
    if (!any) continue;  // uniform: no site in this block
    uint32_t vc[kPer], vm[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int kv = t * kPer + j;
      const int64_t v = kv < nv ? block_voxel(G, b, kv) : -1;
      vc[j] = v >= 0 ? comp[v] : kNone;
      vm[j] = v >= 0 ? voxel_mass(mi, v) : 0u;
    }
    for (uint32_t k = k0; k < k1; ++k) {
      const uint32_t nb = nb_pair[k];
      if (nb == 0) continue;  // uniform across the workgroup
      const uint32_t c = pair_comp[k];
      const unsigned long long mb = pair_mass[k];
      const uint32_t so = soff_pair[k];
      if (mb == 0) {
        if (t == 0 && so < cap) sites[so] = comp_first[c];
        continue;
      }
      unsigned long long run = 0, loc[kPer];
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        run += vc[j] == c ? vm[j] : 0u;
        loc[j] = run;
      }
      unsigned long long inc = run;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const unsigned long long x = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += x;
      }
      if (lane == kWave - 1) wtot[wid] = inc;
      __syncthreads();
      unsigned long long before = inc - run;
      for (int q = 0; q < wid; ++q) before += wtot[q];
#pragma unroll
      for (int j = 0; j < kPer; ++j) cum[t * kPer + j] = before + loc[j];
      __syncthreads();
      U4 ctr;
      ctr.v[0] = (uint32_t)b;
      ctr.v[1] = c;
      ctr.v[2] = 0u;
      ctr.v[3] = 0u;
      const U4 rnd = philox4x32_10(ctr, key_lo, key_hi);
      const unsigned long long o = ((unsigned long long)rnd.v[0] | ((unsigned long long)rnd.v[1] << 32)) % mb;
      const unsigned long long qm = mb / nb, rm = mb % nb;
      for (uint32_t j = t; j < nb; j += kSeedThreads) {
        // p_j = floor((o + j mb) / nb) without 128-bit products
        const unsigned long long p = (unsigned long long)j * qm + (o + (unsigned long long)j * rm) / nb;
        // first voxel whose cumulative mass exceeds p
        int lo = 0, hi = kBlockCap - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (cum[mid] > p)
            hi = mid;
          else
            lo = mid + 1;
        }
        const int64_t v = block_voxel(G, b, lo);
        if (so + j < cap) sites[so + j] = (uint32_t)v;
      }
      __syncthreads();
    }
  }
}

struct SeedWork {
  uint32_t *pcnt, *poff, *err;
  unsigned long long *bmass, *total;
  uint32_t *pair_comp, *pair_block;
  unsigned long long *pair_mass;
  uint32_t *val_a, *val_b, *pos;
  uint8_t *digit;
  void *scratch;
  size_t scratch_bytes;
  uint32_t *scomp, *snb, *ssoff, *cbeg, *cend, *nb_pair, *soff_pair;
  unsigned long long *smass, *srem;
};

template <class A>
void seed_layout(A &a, const SeedGeom &G, uint32_t n_comp, uint32_t cap_pairs, SeedWork *W) {
  const size_t nb = (size_t)G.nblocks;
  const size_t P = cap_pairs ? cap_pairs : 1;
  auto pcnt = a.template take<uint32_t>(nb + 1);
  auto poff = a.template take<uint32_t>(nb + 1);
  auto err = a.template take<uint32_t>(1);
  auto bmass = a.template take<unsigned long long>(nb);
  auto total = a.template take<unsigned long long>(1);
  auto pc = a.template take<uint32_t>(P);
  auto pb = a.template take<uint32_t>(P);
  auto pm = a.template take<unsigned long long>(P);
  auto va = a.template take<uint32_t>(P);
  auto vb = a.template take<uint32_t>(P);
  auto pos = a.template take<uint32_t>(P);
  auto dig = a.template take<uint8_t>(P);
  const size_t sb = std::max(StableSort8::workspace((int64_t)P), ScanU32::workspace((int64_t)std::max(P, nb)));
  auto scr = a.template take<uint8_t>(sb);
  auto sc = a.template take<uint32_t>(P);
  auto snb = a.template take<uint32_t>(P + 1);
  auto sso = a.template take<uint32_t>(P + 1);
  auto cb = a.template take<uint32_t>(n_comp ? n_comp : 1);
  auto ce = a.template take<uint32_t>(n_comp ? n_comp : 1);
  auto nbp = a.template take<uint32_t>(P);
  auto sop = a.template take<uint32_t>(P);
  auto sm = a.template take<unsigned long long>(P);
  auto sr = a.template take<unsigned long long>(P);
  if (W) {
    W->pcnt = pcnt;
    W->poff = poff;
    W->err = err;
    W->bmass = bmass;
    W->total = total;
    W->pair_comp = pc;
    W->pair_block = pb;
    W->pair_mass = pm;
    W->val_a = va;
    W->val_b = vb;
    W->pos = pos;
    W->digit = dig;
    W->scratch = scr;
    W->scratch_bytes = sb;
    W->scomp = sc;
    W->snb = snb;
    W->ssoff = sso;
    W->cbeg = cb;
    W->cend = ce;
    W->nb_pair = nbp;
    W->soff_pair = sop;
    W->smass = sm;
    W->srem = sr;
  }
}

unsigned blocks_for_n(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

}  // namespace
}  // namespace lsrvt

using namespace lsrvt;

extern "C" size_t lsrvt_seed_workspace(lsrvt_dims dims, uint32_t n_comp, int32_t block, uint32_t cap_pairs) {
  Geom g;
  if (make_geom(dims, g) != LSRVT_OK || block < 1 || block > kMaxBlockEdge || cap_pairs == 0) return 0;
  SeedGeom G = seed_geom(g, block);
  Sizer sz;
  seed_layout(sz, G, n_comp, cap_pairs, nullptr);
  return sz.off;
}

extern "C" int32_t lsrvt_seed(const uint32_t *d_comp, const uint32_t *d_comp_first, lsrvt_dims dims, uint32_t n_comp,
                              const uint16_t *d_weights,
                              const uint32_t *d_mass_lut, uint32_t rho, int32_t block, uint64_t seed,
                              uint32_t cap_pairs, uint32_t *d_sites, uint32_t cap_sites, uint32_t *h_n_sites,
                              uint32_t *h_n_pairs, void *d_work, size_t work_bytes, void *stream) {
  Geom g;
  int32_t rc = make_geom(dims, g);
  if (rc) return rc;
  if (!d_comp || !d_comp_first || rho == 0 || block < 1 || block > kMaxBlockEdge || cap_pairs == 0 || n_comp == 0 ||
      (cap_sites > 0 && !d_sites) || (d_mass_lut && !d_weights))
    return LSRVT_EINVAL;
  if (h_n_sites) *h_n_sites = 0;
  if (h_n_pairs) *h_n_pairs = 0;
  const SeedGeom G = seed_geom(g, block);
  const size_t need = lsrvt_seed_workspace(dims, n_comp, block, cap_pairs);
  if ((rc = check_work(d_work, work_bytes, need))) return rc;
  Carve cv(d_work, work_bytes);
  SeedWork W;
  seed_layout(cv, G, n_comp, cap_pairs, &W);
  if (!cv.ok) return LSRVT_EWORKSPACE;
  hipStream_t s = as_stream(stream);
  const MassIn mi{d_weights, d_mass_lut};
  const unsigned gb = (unsigned)std::min<int64_t>(G.nblocks, 65535);
  if ((rc = fill<uint32_t>(W.err, 1, 0u, s))) return rc;
  // pairs per block, block masses, total mass
  hipLaunchKernelGGL(k_seed_blocks<0>, dim3(gb), dim3(kSeedThreads), 0, s, d_comp, G, n_comp, mi, W.pcnt, W.bmass,
                     nullptr, nullptr, nullptr, nullptr, W.err);
  hipLaunchKernelGGL(k_seed_total, dim3(1), dim3(kSeedThreads), 0, s, W.bmass, G.nblocks, W.total);
  LSRVT_LAUNCHED();
  if ((rc = ScanU32::run(W.pcnt, G.nblocks, W.poff, W.scratch, W.scratch_bytes, s))) return rc;
  uint32_t hdr[2] = {0, 0};
  LSRVT_HIP(hipMemcpyAsync(&hdr[0], W.poff + G.nblocks, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  LSRVT_HIP(hipMemcpyAsync(&hdr[1], W.err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  LSRVT_HIP(hipStreamSynchronize(s));
  if (hdr[1] & 1u) return LSRVT_EINVAL;
  const uint32_t P = hdr[0];
  if (h_n_pairs) *h_n_pairs = P;
  if (P > cap_pairs) return LSRVT_ECAPACITY;
  hipLaunchKernelGGL(k_seed_blocks<1>, dim3(gb), dim3(kSeedThreads), 0, s, d_comp, G, n_comp, mi, W.pcnt, W.bmass,
                     W.poff, W.pair_comp, W.pair_block, W.pair_mass, W.err);
  // stable radix sort of the pairs by component (block order is kept)
  hipLaunchKernelGGL(k_seed_iota, dim3(blocks_for_n(P)), dim3(256), 0, s, W.val_a, (int64_t)P);
  LSRVT_LAUNCHED();
  uint32_t *cur = W.val_a, *other = W.val_b;
  for (int p = 0; p < 4 && (p == 0 || (n_comp - 1) >> (8 * p)); ++p) {
    hipLaunchKernelGGL(k_seed_digit, dim3(blocks_for_n(P)), dim3(256), 0, s, cur, (int64_t)P, W.pair_comp, 8 * p,
                       W.digit);
    LSRVT_LAUNCHED();
    if ((rc = StableSort8::run(W.digit, P, W.pos, nullptr, W.scratch, W.scratch_bytes, s))) return rc;
    hipLaunchKernelGGL(k_seed_scatter, dim3(blocks_for_n(P)), dim3(256), 0, s, cur, W.pos, (int64_t)P, other);
    LSRVT_LAUNCHED();
    std::swap(cur, other);
  }
  if ((rc = fill<uint32_t>(W.cbeg, n_comp, 0u, s))) return rc;
  if ((rc = fill<uint32_t>(W.cend, n_comp, 0u, s))) return rc;
  hipLaunchKernelGGL(k_seed_sorted, dim3(blocks_for_n(P)), dim3(256), 0, s, cur, (int64_t)P, W.pair_comp,
                     W.pair_mass, W.scomp, W.smass, W.cbeg, W.cend);
  hipLaunchKernelGGL(k_seed_apportion, dim3(grid_for(n_comp, kSeedThreads / kWave, 65535)), dim3(kSeedThreads), 0,
                     s, n_comp, W.cbeg, W.cend, cur, W.smass, W.total, g.n, rho, W.srem, W.snb,
                     W.err);
  LSRVT_LAUNCHED();
  if ((rc = ScanU32::run(W.snb, P, W.ssoff, W.scratch, W.scratch_bytes, s))) return rc;
  uint32_t S = 0;
  LSRVT_HIP(hipMemcpyAsync(&S, W.ssoff + P, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  LSRVT_HIP(hipMemcpyAsync(&hdr[1], W.err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  LSRVT_HIP(hipStreamSynchronize(s));
  if (hdr[1] & 1u) return LSRVT_EINVAL;
  if (hdr[1]) return LSRVT_ELIMIT;
  if (h_n_sites) *h_n_sites = S;
  if (S > cap_sites) return LSRVT_ECAPACITY;
  hipLaunchKernelGGL(k_seed_unsort, dim3(blocks_for_n(P)), dim3(256), 0, s, cur, (int64_t)P, W.snb, W.ssoff,
                     W.nb_pair, W.soff_pair);
  hipLaunchKernelGGL(k_seed_place, dim3(gb), dim3(kSeedThreads), 0, s, d_comp, G, mi, W.poff, W.pair_comp,
                     W.pair_mass, d_comp_first, W.nb_pair, W.soff_pair, (uint32_t)seed, (uint32_t)(seed >> 32),
                     d_sites, cap_sites);
  LSRVT_LAUNCHED();
  return LSRVT_OK;
}
