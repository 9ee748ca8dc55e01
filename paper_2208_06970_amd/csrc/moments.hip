// Joint moments up to fourth order of every cell, component and band: the
// centred sums M2 (covariance), M3 (coskewness) and M4 (cokurtosis) that the
// joint plots compare between the raw data and the fitted distribution
// models (Sec. 4.4), merged up the hierarchy of Sec. 3.2.4 / Fig. 5.
//
// Cells: the voxels of a cell are one range of the structured layout; one
// workgroup per cell stages 256 voxels at a time in LDS as float64 offsets
// d = x - x(site) and each thread accumulates the raw sums of one or two
// "units" (S1_i, S2_ij, S3_ijk, S4_ijkl over index tuples in lexicographic
// order).  The raw sums about the site value become centred sums with the
// mean offset a = S1 / n:
//   M2_ij   = S2_ij - n a_i a_j
//   M3_ijk  = S3_ijk - (a_i S2_jk + a_j S2_ik + a_k S2_ij) + 2 n a_i a_j a_k
//   M4_ijkl = S4_ijkl - sum over the 4 indices of a_x S3_(other three)
//             + sum over the 6 index pairs of a_x a_y S2_(other two)
//             - 3 n a_i a_j a_k a_l.
// Components and bands: pairwise merges (Pebay, "Formulas for robust,
// one-pass parallel computation of covariances and arbitrary-order
// statistical moments", 2008): for parts A, B with n = nA + nB and
// delta = mean_B - mean_A,
//   M2_ab   = M2A + M2B + nA nB / n d_a d_b
//   M3_abc  = M3A + M3B + nA nB (nA - nB) / n^2 d_a d_b d_c
//             + 1/n sum over the 3 indices x of d_x (nA M2B - nB M2A)_(other two)
//   M4_abcd = M4A + M4B + nA nB (nA^2 - nA nB + nB^2) / n^3 d_a d_b d_c d_d
//             + 1/n^2 sum over the 6 index pairs {x,y} of d_x d_y (nA^2 M2B + nB^2 M2A)_(other two)
//             + 1/n sum over the 4 indices x of d_x (nA M3B - nB M3A)_(other three)
// in a fixed order (cells of a component by site id, components of a band by
// id), in chunks of kMergeChunk members merged one wave each and then the
// chunk results in order.  Everything is float64.
#include <algorithm>

#include "layout.h"

namespace lsrvt {
namespace {

constexpr int kMomMaxVars = 8;
constexpr int kMomThreads = 256;
constexpr int kMaxUnits = 512;  // m + P2 + P3 + P4 <= 494 for m = 8
constexpr int kMergeChunk = 128;

struct MomShape {
  int m, P2, P3, P4, U;  // U = m + P2 + P3 + P4 raw units
};

MomShape mom_shape(int m) {
  MomShape s;
  s.m = m;
  s.P2 = m * (m + 1) / 2;
  s.P3 = m * (m + 1) * (m + 2) / 6;
  s.P4 = m * (m + 1) * (m + 2) * (m + 3) / 24;
  s.U = m + s.P2 + s.P3 + s.P4;
  return s;
}

// Tables built on the device by one thread: code[u] = order | i << 4 | j << 8
// | k << 12 | l << 16 of raw unit u (units of order 1, then 2, 3, 4, each in
// lexicographic order of i <= j <= k <= l), and the packed position of every
// sorted pair and triple.
struct MomTables {
  uint32_t *code;  // [U]
  uint16_t *idx2;  // [m][m]
  uint16_t *idx3;  // [m][m][m]
};

__global__ void k_mom_tables(MomShape S, MomTables T) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const int m = S.m;
  int u = 0;
  for (int i = 0; i < m; ++i) T.code[u++] = 1u | (uint32_t)i << 4;
  int p = 0;
  for (int i = 0; i < m; ++i)
    for (int j = i; j < m; ++j) {
      T.idx2[i * m + j] = (uint16_t)p++;
      T.code[u++] = 2u | (uint32_t)i << 4 | (uint32_t)j << 8;
    }
  p = 0;
  for (int i = 0; i < m; ++i)
    for (int j = i; j < m; ++j)
      for (int k = j; k < m; ++k) {
        T.idx3[(i * m + j) * m + k] = (uint16_t)p++;
        T.code[u++] = 3u | (uint32_t)i << 4 | (uint32_t)j << 8 | (uint32_t)k << 12;
      }
  for (int i = 0; i < m; ++i)
    for (int j = i; j < m; ++j)
      for (int k = j; k < m; ++k)
        for (int l = k; l < m; ++l)
          T.code[u++] = 4u | (uint32_t)i << 4 | (uint32_t)j << 8 | (uint32_t)k << 12 | (uint32_t)l << 16;
}

struct MomOut {
  uint64_t *n;
  double *mean, *m2, *m3, *m4;
};

__device__ __forceinline__ int cidx(uint32_t code, int q) { return (int)((code >> (4 + 4 * q)) & 15u); }

// sorted-tuple lookups (a <= b <= c)
__device__ __forceinline__ int p2(const uint16_t *idx2, int m, int a, int b) { return idx2[a * m + b]; }
__device__ __forceinline__ int p3(const uint16_t *idx3, int m, int a, int b, int c) {
  return idx3[(a * m + b) * m + c];
}

// One workgroup per cell (rank r of the layout): raw sums about the site
// value, then the centred sums, written at the cell's site id.
__global__ __launch_bounds__(kMomThreads) void k_mom_cells(const uint32_t *__restrict__ perm,
                                                           const uint32_t *__restrict__ cell_off,
                                                           const uint32_t *__restrict__ order,
                                                           const uint32_t *__restrict__ sites, uint32_t S,
                                                           const float *__restrict__ vars, int64_t N, MomShape sh,
                                                           MomTables T, MomOut out) {
  __shared__ double dch[kMomThreads * kMomMaxVars];
  __shared__ double raw[kMaxUnits];
  __shared__ uint16_t i2[kMomMaxVars * kMomMaxVars], i3[kMomMaxVars * kMomMaxVars * kMomMaxVars];
  const int t = threadIdx.x;
  const int m = sh.m;
  for (int i = t; i < m * m; i += kMomThreads) i2[i] = T.idx2[i];
  for (int i = t; i < m * m * m; i += kMomThreads) i3[i] = T.idx3[i];
  const uint32_t c0 = t < sh.U ? T.code[t] : 0u;
  const uint32_t c1 = t + kMomThreads < sh.U ? T.code[t + kMomThreads] : 0u;
  for (uint32_t r = blockIdx.x; r < S; r += gridDim.x) {
    const uint32_t lo = cell_off[r], hi = cell_off[r + 1];
    const uint32_t site = order[r];
    const uint32_t sv = sites[site];
    double acc0 = 0.0, acc1 = 0.0;
    for (uint32_t base = lo; base < hi; base += kMomThreads) {
      const uint32_t cnt = min((uint32_t)kMomThreads, hi - base);
      __syncthreads();
      if ((uint32_t)t < cnt) {
        const uint32_t v = perm[base + t];
        for (int j = 0; j < m; ++j)
          dch[t * kMomMaxVars + j] = (double)vars[(int64_t)j * N + v] - (double)vars[(int64_t)j * N + sv];
      }
      __syncthreads();
      for (uint32_t i = 0; i < cnt; ++i) {
        const double *d = dch + i * kMomMaxVars;
        if (c0) {
          double p = d[cidx(c0, 0)];
          const int o = (int)(c0 & 15u);
          if (o > 1) p *= d[cidx(c0, 1)];
          if (o > 2) p *= d[cidx(c0, 2)];
          if (o > 3) p *= d[cidx(c0, 3)];
          acc0 += p;
        }
        if (c1) {
          double p = d[cidx(c1, 0)];
          const int o = (int)(c1 & 15u);
          if (o > 1) p *= d[cidx(c1, 1)];
          if (o > 2) p *= d[cidx(c1, 2)];
          if (o > 3) p *= d[cidx(c1, 3)];
          acc1 += p;
        }
      }
    }
    if (t < sh.U) raw[t] = acc0;
    if (t + kMomThreads < sh.U) raw[t + kMomThreads] = acc1;
    __syncthreads();
    const double n = (double)(hi - lo);
    const double *S1 = raw, *S2 = raw + m, *S3 = raw + m + sh.P2, *S4 = raw + m + sh.P2 + sh.P3;
    // mean offsets a_j = S1_j / n (0 for an empty cell)
    auto a = [&](int j) { return hi > lo ? S1[j] / n : 0.0; };
    for (int u = t; u < sh.U; u += kMomThreads) {
      const uint32_t code = T.code[u];
      const int o = (int)(code & 15u);
      const int i = cidx(code, 0), j = cidx(code, 1), k = cidx(code, 2), l = cidx(code, 3);
      if (o == 1) {
        out.mean[(int64_t)site * m + i] = (double)vars[(int64_t)i * N + sv] + a(i);
      } else if (o == 2) {
        const int q = u - m;
        out.m2[(int64_t)site * sh.P2 + q] = S2[q] - n * a(i) * a(j);
      } else if (o == 3) {
        const int q = u - m - sh.P2;
        const double v = S3[q] - (a(i) * S2[p2(i2, m, j, k)] + a(j) * S2[p2(i2, m, i, k)] + a(k) * S2[p2(i2, m, i, j)]) +
                         2.0 * n * a(i) * a(j) * a(k);
        out.m3[(int64_t)site * sh.P3 + q] = v;
      } else {
        const int q = u - m - sh.P2 - sh.P3;
        double v = S4[q];
        v -= a(i) * S3[p3(i3, m, j, k, l)] + a(j) * S3[p3(i3, m, i, k, l)] + a(k) * S3[p3(i3, m, i, j, l)] +
             a(l) * S3[p3(i3, m, i, j, k)];
        v += a(i) * a(j) * S2[p2(i2, m, k, l)] + a(i) * a(k) * S2[p2(i2, m, j, l)] + a(i) * a(l) * S2[p2(i2, m, j, k)] +
             a(j) * a(k) * S2[p2(i2, m, i, l)] + a(j) * a(l) * S2[p2(i2, m, i, k)] + a(k) * a(l) * S2[p2(i2, m, i, j)];
        v -= 3.0 * n * a(i) * a(j) * a(k) * a(l);
        out.m4[(int64_t)site * sh.P4 + q] = v;
      }
    }
    if (t == 0) out.n[site] = (uint64_t)(hi - lo);
    if (hi == lo)
      for (int j = t; j < m; j += kMomThreads) out.mean[(int64_t)site * m + j] = 0.0;
    __syncthreads();
  }
}

// Moments of one part, held in LDS by one wave: n, mean[m], M2[P2], M3[P3], M4[P4].
struct PartView {
  double *n, *mean, *m2, *m3, *m4;
};

__device__ __forceinline__ PartView part_at(double *base, const MomShape &sh) {
  PartView p;
  p.n = base;
  p.mean = base + 1;
  p.m2 = p.mean + sh.m;
  p.m3 = p.m2 + sh.P2;
  p.m4 = p.m3 + sh.P3;
  return p;
}

// C = merge(A, B) over the lanes of one wave (C distinct from A and B).
__device__ void merge_parts(const PartView &A, const PartView &B, const PartView &C, const MomShape &sh,
                            const uint32_t *code, const uint16_t *i2, const uint16_t *i3) {
  const int lane = lane_id();
  const int m = sh.m;
  const double nA = *A.n, nB = *B.n;
  if (nB == 0.0 || nA == 0.0) {
    const PartView &X = nB == 0.0 ? A : B;
    const int len = 1 + sh.U;
    for (int q = lane; q < len; q += kWave) C.n[q] = X.n[q];
    return;
  }
  const double n = nA + nB;
  auto d = [&](int x) { return B.mean[x] - A.mean[x]; };
  for (int u = lane; u < sh.U; u += kWave) {
    const uint32_t cd = code[u];
    const int o = (int)(cd & 15u);
    const int a = cidx(cd, 0), b = cidx(cd, 1), c = cidx(cd, 2), e = cidx(cd, 3);
    if (o == 1) {
      C.mean[a] = A.mean[a] + d(a) * (nB / n);
    } else if (o == 2) {
      const int q = u - m;
      C.m2[q] = A.m2[q] + B.m2[q] + nA * nB / n * d(a) * d(b);
    } else if (o == 3) {
      const int q = u - m - sh.P2;
      auto w2 = [&](int x, int y) {
        const int k = p2(i2, m, x, y);
        return nA * B.m2[k] - nB * A.m2[k];
      };
      C.m3[q] = A.m3[q] + B.m3[q] + nA * nB * (nA - nB) / (n * n) * d(a) * d(b) * d(c) +
                (d(a) * w2(b, c) + d(b) * w2(a, c) + d(c) * w2(a, b)) / n;
    } else {
      const int q = u - m - sh.P2 - sh.P3;
      auto v2 = [&](int x, int y) {
        const int k = p2(i2, m, x, y);
        return nA * nA * B.m2[k] + nB * nB * A.m2[k];
      };
      auto v3 = [&](int x, int y, int z) {
        const int k = p3(i3, m, x, y, z);
        return nA * B.m3[k] - nB * A.m3[k];
      };
      const double t4 = nA * nB * (nA * nA - nA * nB + nB * nB) / (n * n * n) * d(a) * d(b) * d(c) * d(e);
      const double t2 = (d(a) * d(b) * v2(c, e) + d(a) * d(c) * v2(b, e) + d(a) * d(e) * v2(b, c) +
                         d(b) * d(c) * v2(a, e) + d(b) * d(e) * v2(a, c) + d(c) * d(e) * v2(a, b)) /
                        (n * n);
      const double t3 = (d(a) * v3(b, c, e) + d(b) * v3(a, c, e) + d(c) * v3(a, b, e) + d(e) * v3(a, b, c)) / n;
      C.m4[q] = A.m4[q] + B.m4[q] + t4 + t2 + t3;
    }
  }
  if (lane == 0) *C.n = n;
}

// Group inputs: members of group g are member_id(lo + k) for k < hi - lo.
struct MergeIn {
  const uint64_t *n;  // member arrays in the MomOut layout
  const double *mean, *m2, *m3, *m4;
  const uint32_t *map;  // member index -> row (null: identity)
};

__device__ void load_part(const MergeIn &in, uint32_t row, const PartView &P, const MomShape &sh) {
  const int lane = lane_id();
  if (lane == 0) *P.n = (double)in.n[row];
  for (int q = lane; q < sh.m; q += kWave) P.mean[q] = in.mean[(int64_t)row * sh.m + q];
  for (int q = lane; q < sh.P2; q += kWave) P.m2[q] = in.m2[(int64_t)row * sh.P2 + q];
  for (int q = lane; q < sh.P3; q += kWave) P.m3[q] = in.m3[(int64_t)row * sh.P3 + q];
  for (int q = lane; q < sh.P4; q += kWave) P.m4[q] = in.m4[(int64_t)row * sh.P4 + q];
}

__device__ void store_part(const MomOut &out, uint32_t row, const PartView &P, const MomShape &sh) {
  const int lane = lane_id();
  if (lane == 0) out.n[row] = (uint64_t)*P.n;
  for (int q = lane; q < sh.m; q += kWave) out.mean[(int64_t)row * sh.m + q] = P.mean[q];
  for (int q = lane; q < sh.P2; q += kWave) out.m2[(int64_t)row * sh.P2 + q] = P.m2[q];
  for (int q = lane; q < sh.P3; q += kWave) out.m3[(int64_t)row * sh.P3 + q] = P.m3[q];
  for (int q = lane; q < sh.P4; q += kWave) out.m4[(int64_t)row * sh.P4 + q] = P.m4[q];
}

constexpr int kPartDoubles = 1 + kMaxUnits;

// One wave per job: merges members [lo, hi) of the job in order into row
// `dst` of `out`.  Job j: group = job_group[j], members
// [job_lo[j], job_hi[j]).
__global__ __launch_bounds__(kMomThreads) void k_mom_merge(uint32_t n_jobs, const uint32_t *job_lo,
                                                           const uint32_t *job_hi, MergeIn in, MomOut out,
                                                           MomShape sh, MomTables T) {
  __shared__ double buf[kMomThreads / kWave][3][kPartDoubles];
  __shared__ uint16_t i2[kMomMaxVars * kMomMaxVars], i3[kMomMaxVars * kMomMaxVars * kMomMaxVars];
  __shared__ uint32_t code[kMaxUnits];
  const int t = threadIdx.x, w = t / kWave, lane = lane_id();
  const int m = sh.m;
  for (int i = t; i < m * m; i += kMomThreads) i2[i] = T.idx2[i];
  for (int i = t; i < m * m * m; i += kMomThreads) i3[i] = T.idx3[i];
  for (int i = t; i < sh.U; i += kMomThreads) code[i] = T.code[i];
  __syncthreads();
  const uint32_t waves = gridDim.x * (kMomThreads / kWave);
  for (uint32_t j = blockIdx.x * (kMomThreads / kWave) + w; j < n_jobs; j += waves) {
    PartView acc = part_at(buf[w][0], sh), nxt = part_at(buf[w][1], sh), inc = part_at(buf[w][2], sh);
    if (lane == 0) *acc.n = 0.0;
    for (int q = lane; q < sh.U; q += kWave) acc.mean[q] = 0.0;
    __builtin_amdgcn_wave_barrier();
    for (uint32_t k = job_lo[j]; k < job_hi[j]; ++k) {
      const uint32_t row = in.map ? in.map[k] : k;
      load_part(in, row, inc, sh);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      merge_parts(acc, inc, nxt, sh, code, i2, i3);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const PartView tmp = acc;
      acc = nxt;
      nxt = tmp;
    }
    store_part(out, j, acc, sh);
    __builtin_amdgcn_wave_barrier();
  }
}

// Jobs of the first merge level: chunks of kMergeChunk consecutive members of
// every group (groups given by offsets goff[g] .. goff[g + 1]).
__global__ void k_mom_chunks(const uint32_t *goff, uint32_t G, uint32_t *nchunk) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < G) nchunk[g] = (goff[g + 1] - goff[g] + kMergeChunk - 1) / kMergeChunk;
}

__global__ void k_mom_jobs(const uint32_t *goff, uint32_t G, const uint32_t *coff_chunk, uint32_t *job_lo,
                           uint32_t *job_hi) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const uint32_t lo = goff[g], hi = goff[g + 1];
  uint32_t j = coff_chunk[g];
  for (uint32_t a = lo; a < hi; a += kMergeChunk, ++j) {
    job_lo[j] = a;
    job_hi[j] = min(hi, a + kMergeChunk);
  }
}

// Band ranges of components: comp_band is nondecreasing.
__global__ void k_mom_band_off(const uint8_t *comp_band, uint32_t C, int32_t nb, uint32_t *boff) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b > nb) return;
  uint32_t lo = 0, hi = C;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if ((int)comp_band[mid] < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  boff[b] = lo;
}

struct MomWork {
  LayoutWork lay;
  uint32_t *perm;
  MomTables tab;
  uint32_t *boff, *nchunk, *choff, *job_lo, *job_hi;
  MomOut part;  // first-level merge results (one row per chunk)
  void *scratch;
  size_t scratch_bytes;
};

// Chunks needed by the first merge level of a set of groups.
int64_t chunk_cap(int64_t members, int64_t groups) { return members / kMergeChunk + groups + 1; }

template <class A>
void mom_layout(A &a, const Geom &g, uint32_t S, uint32_t C, int32_t nb, const MomShape &sh, MomWork *W) {
  const int64_t G = (int64_t)std::max<uint32_t>(C, (uint32_t)nb) + 1;
  const int64_t J = chunk_cap((int64_t)S + C, G);
  layout_take(a, g, S, C, W ? &W->lay : nullptr);
  auto perm = a.template take<uint32_t>(g.n);
  auto code = a.template take<uint32_t>(kMaxUnits);
  auto idx2 = a.template take<uint16_t>(kMomMaxVars * kMomMaxVars);
  auto idx3 = a.template take<uint16_t>(kMomMaxVars * kMomMaxVars * kMomMaxVars);
  auto boff = a.template take<uint32_t>((size_t)nb + 1);
  auto nch = a.template take<uint32_t>(G + 1);
  auto cho = a.template take<uint32_t>(G + 1);
  auto jl = a.template take<uint32_t>(J);
  auto jh = a.template take<uint32_t>(J);
  auto pn = a.template take<uint64_t>(J);
  auto pmean = a.template take<double>(J * sh.m);
  auto pm2 = a.template take<double>(J * sh.P2);
  auto pm3 = a.template take<double>(J * sh.P3);
  auto pm4 = a.template take<double>(J * sh.P4);
  if (W) {
    W->perm = perm;
    W->tab.code = code;
    W->tab.idx2 = idx2;
    W->tab.idx3 = idx3;
    W->boff = boff;
    W->nchunk = nch;
    W->choff = cho;
    W->job_lo = jl;
    W->job_hi = jh;
    W->part.n = pn;
    W->part.mean = pmean;
    W->part.m2 = pm2;
    W->part.m3 = pm3;
    W->part.m4 = pm4;
  }
}

size_t mom_scratch(const Geom &g, uint32_t S, uint32_t C, int32_t nb) {
  const int64_t G = (int64_t)std::max<uint32_t>(C, (uint32_t)nb) + 1;
  return std::max(layout_scratch(g, S, C), ScanU32::workspace(G)) + 256;
}

// Two merge levels over groups [goff[g], goff[g + 1]) of members (rows of
// `in`, through `map`), results to rows 0 .. G - 1 of `out`.
int32_t merge_groups(const uint32_t *goff, uint32_t G, const MergeIn &in, const MomOut &out, const MomShape &sh,
                     MomWork &W, hipStream_t s) {
  if (G == 0) return LSRVT_OK;
  int32_t rc;
  hipLaunchKernelGGL(k_mom_chunks, dim3((G + 255) / 256), dim3(256), 0, s, goff, G, W.nchunk);
  LSRVT_LAUNCHED();
  if ((rc = ScanU32::run(W.nchunk, G, W.choff, W.scratch, W.scratch_bytes, s))) return rc;
  uint32_t J = 0;
  {
    const int32_t rc_ = read_words(W.choff + G, 1, &J, s);
    if (rc_) return rc_;
  }
  hipLaunchKernelGGL(k_mom_jobs, dim3((G + 255) / 256), dim3(256), 0, s, goff, G, W.choff, W.job_lo, W.job_hi);
  const unsigned grid1 = (unsigned)std::min<int64_t>(((int64_t)J + 3) / 4, 65535);
  if (J)
    hipLaunchKernelGGL(k_mom_merge, dim3(grid1 ? grid1 : 1), dim3(kMomThreads), 0, s, J, W.job_lo, W.job_hi, in,
                       W.part, sh, W.tab);
  // second level: the chunk results of every group, in order
  MergeIn in2;
  in2.n = W.part.n;
  in2.mean = W.part.mean;
  in2.m2 = W.part.m2;
  in2.m3 = W.part.m3;
  in2.m4 = W.part.m4;
  in2.map = nullptr;
  const unsigned grid2 = (unsigned)std::min<int64_t>(((int64_t)G + 3) / 4, 65535);
  hipLaunchKernelGGL(k_mom_merge, dim3(grid2), dim3(kMomThreads), 0, s, G, W.choff, W.choff + 1, in2, out, sh,
                     W.tab);
  LSRVT_LAUNCHED();
  return LSRVT_OK;
}

bool out_ok(const lsrvt_moments *o) { return o && o->n && o->mean && o->m2 && o->m3 && o->m4; }

}  // namespace
}  // namespace lsrvt

using namespace lsrvt;

extern "C" size_t lsrvt_comoments_workspace(lsrvt_dims dims, uint32_t n_sites, uint32_t n_comp, int32_t n_bands,
                                            int32_t n_vars) {
  Geom g;
  if (make_geom(dims, g) || n_vars < 1 || n_vars > kMomMaxVars || n_bands < 1 || n_bands > 255) return 0;
  const MomShape sh = mom_shape(n_vars);
  Sizer z;
  mom_layout(z, g, n_sites, n_comp, n_bands, sh, nullptr);
  return z.off + mom_scratch(g, n_sites, n_comp, n_bands);
}

extern "C" int32_t lsrvt_comoments(const uint32_t *d_cell, lsrvt_dims dims, const uint32_t *d_sites,
                                   const uint32_t *d_site_comp, uint32_t n_sites, const uint8_t *d_comp_band,
                                   uint32_t n_comp, int32_t n_bands, const float *d_vars, int32_t n_vars,
                                   const lsrvt_moments *cell, const lsrvt_moments *comp, const lsrvt_moments *band,
                                   void *d_work, size_t work_bytes, void *stream) {
  Geom g;
  int32_t rc = make_geom(dims, g);
  if (rc) return rc;
  if (n_vars < 1 || n_vars > kMomMaxVars || n_bands < 1 || n_bands > 255) return LSRVT_EINVAL;
  if (!d_cell || !d_vars || !out_ok(cell) || !out_ok(comp) || !out_ok(band)) return LSRVT_EINVAL;
  if (n_sites && (!d_sites || !d_site_comp)) return LSRVT_EINVAL;
  if (n_comp && !d_comp_band) return LSRVT_EINVAL;
  const size_t need = lsrvt_comoments_workspace(dims, n_sites, n_comp, n_bands, n_vars);
  if ((rc = check_work(d_work, work_bytes, need))) return rc;
  const MomShape sh = mom_shape(n_vars);
  Carve cv(d_work, work_bytes);
  MomWork W;
  mom_layout(cv, g, n_sites, n_comp, n_bands, sh, &W);
  if (!cv.ok) return LSRVT_EWORKSPACE;
  W.scratch = cv.base + cv.off;
  W.scratch_bytes = cv.size - cv.off;
  W.lay.scratch = W.scratch;
  W.lay.scratch_bytes = W.scratch_bytes;
  hipStream_t s = as_stream(stream);
  const uint32_t S = n_sites, C = n_comp;
  hipLaunchKernelGGL(k_mom_tables, dim3(1), dim3(64), 0, s, sh, W.tab);
  LSRVT_LAUNCHED();
  // cells: the layout gives every cell one contiguous voxel range
  if ((rc = layout_sites(d_site_comp, S, C, W.lay, s))) return rc;
  if ((rc = layout_voxels(d_cell, g, S, W.lay, W.perm, s))) return rc;
  const MomOut co{cell->n, cell->mean, cell->m2, cell->m3, cell->m4};
  if (S) {
    hipLaunchKernelGGL(k_mom_cells, dim3((unsigned)std::min<uint32_t>(S, 65535)), dim3(kMomThreads), 0, s, W.perm,
                       W.lay.cell_off, W.lay.order, d_sites, S, d_vars, g.n, sh, W.tab, co);
    LSRVT_LAUNCHED();
  }
  // components: their cells by site id (ranks coff[c] .. coff[c + 1])
  MergeIn cin{cell->n, cell->mean, cell->m2, cell->m3, cell->m4, W.lay.order};
  const MomOut go{comp->n, comp->mean, comp->m2, comp->m3, comp->m4};
  if ((rc = merge_groups(W.lay.coff, C, cin, go, sh, W, s))) return rc;
  // bands: their components by id
  hipLaunchKernelGGL(k_mom_band_off, dim3((n_bands + 1 + 255) / 256), dim3(256), 0, s, d_comp_band, C, n_bands,
                     W.boff);
  LSRVT_LAUNCHED();
  MergeIn bin{comp->n, comp->mean, comp->m2, comp->m3, comp->m4, nullptr};
  const MomOut bo{band->n, band->mean, band->m2, band->m3, band->m4};
  if ((rc = merge_groups(W.boff, (uint32_t)n_bands, bin, bo, sh, W, s))) return rc;
  return LSRVT_OK;
}
