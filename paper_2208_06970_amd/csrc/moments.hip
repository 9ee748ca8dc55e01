// Joint moments up to fourth order of every cell, component and band: the
// centred sums M2 (covariance), M3 (coskewness) and M4 (cokurtosis) that the
// joint plots compare between the raw data and the fitted distribution
// models (Sec. 4.4), merged up the hierarchy of Sec. 3.2.4 / Fig. 5.  Up to
// 18 variables: 7314 sums of orders 1 to 4 per unit.
//
// Cells: the voxels of a cell are one range of the structured layout.  The
// raw sums about the site value (S1_i, S2_ij, S3_ijk, S4_ijkl over index
// tuples in lexicographic order, the "units") are taken in passes of 1024
// units: one workgroup per (cell, pass) stages 256 voxels at a time in LDS
// as float64 offsets d = x - x(site) and each thread sums four units.  The
// raw sums, written to the cell's output rows, then become centred sums in
// place with the mean offset a = S1 / n (k_mom_center).
// Components and bands: pairwise merges (Pebay, "Formulas for robust,
// one-pass parallel computation of covariances and arbitrary-order
// statistical moments", 2008; the formulas at k_mom_merge) in a fixed order
// (cells of a component by site id, components of a band by id), in chunks
// of kMergeChunk members merged in place by one workgroup each and then the
// chunk results in order.  Everything is float64.
#include <algorithm>

#include "layout.h"

namespace lsrvt {
namespace {

constexpr int kMomMaxVars = 18;  // 7314 moments of orders 1..4 per unit at m = 18
constexpr int kMomThreads = 256;
constexpr int kMomUPT = 4;                            // raw-sum units per thread and cell pass
constexpr int kMomChunk = kMomThreads * kMomUPT;      // units per cell pass
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

// Tables built on the device by one thread: code[u] = order | i << 4 | j << 9
// | k << 14 | l << 19 of raw unit u (units of order 1, then 2, 3, 4, each in
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
      T.code[u++] = 2u | (uint32_t)i << 4 | (uint32_t)j << 9;
    }
  p = 0;
  for (int i = 0; i < m; ++i)
    for (int j = i; j < m; ++j)
      for (int k = j; k < m; ++k) {
        T.idx3[(i * m + j) * m + k] = (uint16_t)p++;
        T.code[u++] = 3u | (uint32_t)i << 4 | (uint32_t)j << 9 | (uint32_t)k << 14;
      }
  for (int i = 0; i < m; ++i)
    for (int j = i; j < m; ++j)
      for (int k = j; k < m; ++k)
        for (int l = k; l < m; ++l)
          T.code[u++] = 4u | (uint32_t)i << 4 | (uint32_t)j << 9 | (uint32_t)k << 14 | (uint32_t)l << 19;
}

struct MomOut {
  uint64_t *n;
  double *mean, *m2, *m3, *m4;
};

__device__ __forceinline__ int cidx(uint32_t code, int q) { return (int)((code >> (4 + 5 * q)) & 31u); }

// sorted-tuple lookups (a <= b <= c)
__device__ __forceinline__ int p2(const uint16_t *idx2, int m, int a, int b) { return idx2[a * m + b]; }
__device__ __forceinline__ int p3(const uint16_t *idx3, int m, int a, int b, int c) {
  return idx3[(a * m + b) * m + c];
}

// Raw sums about the site value of every cell (rank r of the layout), units
// [blockIdx.y * kMomChunk, + kMomChunk): the cell's voxels are staged 256 at a
// time in LDS as float64 offsets d = x - x(site); thread t sums the products
// of units u0 + t, u0 + t + 256, ... over the voxels in layout order.  The
// sums go to the cell's rows of the outputs (order 1 to mean, 2 to m2, ...),
// where k_mom_center turns them into centred sums.
__global__ __launch_bounds__(kMomThreads) void k_mom_cells(const uint32_t *__restrict__ perm,
                                                           const uint32_t *__restrict__ cell_off,
                                                           const uint32_t *__restrict__ order,
                                                           const uint32_t *__restrict__ sites, uint32_t S,
                                                           const float *__restrict__ vars, int64_t N, MomShape sh,
                                                           MomTables T, MomOut out) {
  __shared__ double dch[kMomThreads * kMomMaxVars];
  const int t = threadIdx.x;
  const int m = sh.m;
  const int u0 = (int)blockIdx.y * kMomChunk;
  uint32_t cd[kMomUPT];
#pragma unroll
  for (int q = 0; q < kMomUPT; ++q) {
    const int u = u0 + q * kMomThreads + t;
    cd[q] = u < sh.U ? T.code[u] : 0u;
  }
  for (uint32_t r = blockIdx.x; r < S; r += gridDim.x) {
    const uint32_t lo = cell_off[r], hi = cell_off[r + 1];
    const uint32_t site = order[r];
    const uint32_t sv = sites[site];
    double acc[kMomUPT];
#pragma unroll
    for (int q = 0; q < kMomUPT; ++q) acc[q] = 0.0;
    for (uint32_t base = lo; base < hi; base += kMomThreads) {
      const uint32_t cnt = min((uint32_t)kMomThreads, hi - base);
      __syncthreads();
      if ((uint32_t)t < cnt) {
        const uint32_t v = perm[base + t];
        for (int j = 0; j < m; ++j)
          dch[t * m + j] = (double)vars[(int64_t)j * N + v] - (double)vars[(int64_t)j * N + sv];
      }
      __syncthreads();
      for (uint32_t i = 0; i < cnt; ++i) {
        const double *d = dch + i * m;
#pragma unroll
        for (int q = 0; q < kMomUPT; ++q) {
          const uint32_t c = cd[q];
          if (!c) continue;
          double p = d[cidx(c, 0)];
          const int o = (int)(c & 15u);
          if (o > 1) p *= d[cidx(c, 1)];
          if (o > 2) p *= d[cidx(c, 2)];
          if (o > 3) p *= d[cidx(c, 3)];
          acc[q] += p;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kMomUPT; ++q) {
      const int u = u0 + q * kMomThreads + t;
      if (u >= sh.U) continue;
      if (u < m)
        out.mean[(int64_t)site * m + u] = acc[q];
      else if (u < m + sh.P2)
        out.m2[(int64_t)site * sh.P2 + (u - m)] = acc[q];
      else if (u < m + sh.P2 + sh.P3)
        out.m3[(int64_t)site * sh.P3 + (u - m - sh.P2)] = acc[q];
      else
        out.m4[(int64_t)site * sh.P4 + (u - m - sh.P2 - sh.P3)] = acc[q];
    }
  }
}

// The raw sums of every cell about its site value become centred sums with
// the mean offset a = S1 / n, in place, highest order first (each order reads
// only lower orders' raw sums, which are rewritten later):
//   M4_ijkl = S4_ijkl - sum over the 4 indices of a_x S3_(other three)
//             + sum over the 6 index pairs of a_x a_y S2_(other two)
//             - 3 n a_i a_j a_k a_l
//   M3_ijk  = S3_ijk - (a_i S2_jk + a_j S2_ik + a_k S2_ij) + 2 n a_i a_j a_k
//   M2_ij   = S2_ij - n a_i a_j
//   mean_i  = x_i(site) + a_i
// One workgroup per cell.
__global__ __launch_bounds__(kMomThreads) void k_mom_center(const uint32_t *__restrict__ cell_off,
                                                            const uint32_t *__restrict__ order,
                                                            const uint32_t *__restrict__ sites, uint32_t S,
                                                            const float *__restrict__ vars, int64_t N, MomShape sh,
                                                            MomTables T, MomOut out) {
  __shared__ uint16_t i2[kMomMaxVars * kMomMaxVars], i3[kMomMaxVars * kMomMaxVars * kMomMaxVars];
  __shared__ double a_s[kMomMaxVars];
  const int t = threadIdx.x;
  const int m = sh.m;
  for (int i = t; i < m * m; i += kMomThreads) i2[i] = T.idx2[i];
  for (int i = t; i < m * m * m; i += kMomThreads) i3[i] = T.idx3[i];
  for (uint32_t r = blockIdx.x; r < S; r += gridDim.x) {
    const uint32_t lo = cell_off[r], hi = cell_off[r + 1];
    const uint32_t site = order[r];
    const double n = (double)(hi - lo);
    double *mean = out.mean + (int64_t)site * m, *m2 = out.m2 + (int64_t)site * sh.P2,
           *m3 = out.m3 + (int64_t)site * sh.P3, *m4 = out.m4 + (int64_t)site * sh.P4;
    __syncthreads();
    if (t < m) a_s[t] = hi > lo ? mean[t] / n : 0.0;
    __syncthreads();
    auto a = [&](int j) { return a_s[j]; };
    for (int q = t; q < sh.P4; q += kMomThreads) {
      const uint32_t code = T.code[m + sh.P2 + sh.P3 + q];
      const int i = cidx(code, 0), j = cidx(code, 1), k = cidx(code, 2), l = cidx(code, 3);
      double v = m4[q];
      v -= a(i) * m3[p3(i3, m, j, k, l)] + a(j) * m3[p3(i3, m, i, k, l)] + a(k) * m3[p3(i3, m, i, j, l)] +
           a(l) * m3[p3(i3, m, i, j, k)];
      v += a(i) * a(j) * m2[p2(i2, m, k, l)] + a(i) * a(k) * m2[p2(i2, m, j, l)] + a(i) * a(l) * m2[p2(i2, m, j, k)] +
           a(j) * a(k) * m2[p2(i2, m, i, l)] + a(j) * a(l) * m2[p2(i2, m, i, k)] + a(k) * a(l) * m2[p2(i2, m, i, j)];
      v -= 3.0 * n * a(i) * a(j) * a(k) * a(l);
      m4[q] = v;
    }
    __syncthreads();
    for (int q = t; q < sh.P3; q += kMomThreads) {
      const uint32_t code = T.code[m + sh.P2 + q];
      const int i = cidx(code, 0), j = cidx(code, 1), k = cidx(code, 2);
      m3[q] = m3[q] - (a(i) * m2[p2(i2, m, j, k)] + a(j) * m2[p2(i2, m, i, k)] + a(k) * m2[p2(i2, m, i, j)]) +
              2.0 * n * a(i) * a(j) * a(k);
    }
    __syncthreads();
    for (int q = t; q < sh.P2; q += kMomThreads) {
      const uint32_t code = T.code[m + q];
      const int i = cidx(code, 0), j = cidx(code, 1);
      m2[q] = m2[q] - n * a(i) * a(j);
    }
    if (t < m) mean[t] = hi > lo ? (double)vars[(int64_t)t * N + sites[site]] + a(t) : 0.0;
    if (t == 0) out.n[site] = (uint64_t)(hi - lo);
  }
}

// Group inputs: members of group g are member_id(lo + k) for k < hi - lo.
struct MergeIn {
  const uint64_t *n;  // member arrays in the MomOut layout
  const double *mean, *m2, *m3, *m4;
  const uint32_t *map;  // member index -> row (null: identity)
};

// One workgroup per job: members [job_lo[j], job_hi[j]) merged in order into
// row j of `out`, in place (Pebay's pairwise formulas; A the running result,
// B the next member, n = nA + nB, d = mean_B - mean_A):
//   M4_abcd += M4B + nA nB (nA^2 - nA nB + nB^2) / n^3 d_a d_b d_c d_d
//              + 1/n^2 sum over the 6 index pairs {x,y} of d_x d_y (nA^2 M2B + nB^2 M2A)_(other two)
//              + 1/n sum over the 4 indices x of d_x (nA M3B - nB M3A)_(other three)
//   M3_abc  += M3B + nA nB (nA - nB) / n^2 d_a d_b d_c
//              + 1/n sum over the 3 indices x of d_x (nA M2B - nB M2A)_(other two)
//   M2_ab   += M2B + nA nB / n d_a d_b
//   mean_a  += d_a nB / n
// highest order first, so every order still reads the lower orders of A
// before the merge.
__global__ __launch_bounds__(kMomThreads) void k_mom_merge(uint32_t n_jobs, const uint32_t *job_lo,
                                                           const uint32_t *job_hi, MergeIn in, MomOut out,
                                                           MomShape sh, MomTables T) {
  __shared__ uint16_t i2[kMomMaxVars * kMomMaxVars], i3[kMomMaxVars * kMomMaxVars * kMomMaxVars];
  __shared__ double d_s[kMomMaxVars];
  const int t = threadIdx.x;
  const int m = sh.m;
  for (int i = t; i < m * m; i += kMomThreads) i2[i] = T.idx2[i];
  for (int i = t; i < m * m * m; i += kMomThreads) i3[i] = T.idx3[i];
  const int len = sh.U;  // mean, m2, m3, m4 of a row, as one index space
  for (uint32_t j = blockIdx.x; j < n_jobs; j += gridDim.x) {
    double *A1 = out.mean + (int64_t)j * m, *A2 = out.m2 + (int64_t)j * sh.P2, *A3 = out.m3 + (int64_t)j * sh.P3,
           *A4 = out.m4 + (int64_t)j * sh.P4;
    auto copy_in = [&](uint32_t row) {
      for (int q = t; q < len; q += kMomThreads) {
        if (q < m)
          A1[q] = in.mean[(int64_t)row * m + q];
        else if (q < m + sh.P2)
          A2[q - m] = in.m2[(int64_t)row * sh.P2 + q - m];
        else if (q < m + sh.P2 + sh.P3)
          A3[q - m - sh.P2] = in.m3[(int64_t)row * sh.P3 + q - m - sh.P2];
        else
          A4[q - m - sh.P2 - sh.P3] = in.m4[(int64_t)row * sh.P4 + q - m - sh.P2 - sh.P3];
      }
    };
    const uint32_t lo = job_lo[j], hi = job_hi[j];
    __syncthreads();
    uint64_t nAi = 0;
    if (hi > lo) {
      const uint32_t row = in.map ? in.map[lo] : lo;
      copy_in(row);
      nAi = in.n[row];
    } else {
      for (int q = t; q < len; q += kMomThreads) {
        if (q < m)
          A1[q] = 0.0;
        else if (q < m + sh.P2)
          A2[q - m] = 0.0;
        else if (q < m + sh.P2 + sh.P3)
          A3[q - m - sh.P2] = 0.0;
        else
          A4[q - m - sh.P2 - sh.P3] = 0.0;
      }
    }
    __syncthreads();
    for (uint32_t k = lo + 1; k < hi; ++k) {
      const uint32_t row = in.map ? in.map[k] : k;
      const uint64_t nBi = in.n[row];
      if (nBi == 0) continue;  // uniform
      if (nAi == 0) {
        copy_in(row);
        nAi = nBi;
        __syncthreads();
        continue;
      }
      const double nA = (double)nAi, nB = (double)nBi, n = nA + nB;
      const double *B1 = in.mean + (int64_t)row * m, *B2 = in.m2 + (int64_t)row * sh.P2,
                   *B3 = in.m3 + (int64_t)row * sh.P3, *B4 = in.m4 + (int64_t)row * sh.P4;
      if (t < m) d_s[t] = B1[t] - A1[t];
      __syncthreads();
      auto d = [&](int x) { return d_s[x]; };
      for (int q = t; q < sh.P4; q += kMomThreads) {
        const uint32_t cd = T.code[m + sh.P2 + sh.P3 + q];
        const int a = cidx(cd, 0), b = cidx(cd, 1), c = cidx(cd, 2), e = cidx(cd, 3);
        auto v2 = [&](int x, int y) {
          const int kk = p2(i2, m, x, y);
          return nA * nA * B2[kk] + nB * nB * A2[kk];
        };
        auto v3 = [&](int x, int y, int z) {
          const int kk = p3(i3, m, x, y, z);
          return nA * B3[kk] - nB * A3[kk];
        };
        const double t4 = nA * nB * (nA * nA - nA * nB + nB * nB) / (n * n * n) * d(a) * d(b) * d(c) * d(e);
        const double t2 = (d(a) * d(b) * v2(c, e) + d(a) * d(c) * v2(b, e) + d(a) * d(e) * v2(b, c) +
                           d(b) * d(c) * v2(a, e) + d(b) * d(e) * v2(a, c) + d(c) * d(e) * v2(a, b)) /
                          (n * n);
        const double t3 = (d(a) * v3(b, c, e) + d(b) * v3(a, c, e) + d(c) * v3(a, b, e) + d(e) * v3(a, b, c)) / n;
        A4[q] = A4[q] + B4[q] + t4 + t2 + t3;
      }
      __syncthreads();
      for (int q = t; q < sh.P3; q += kMomThreads) {
        const uint32_t cd = T.code[m + sh.P2 + q];
        const int a = cidx(cd, 0), b = cidx(cd, 1), c = cidx(cd, 2);
        auto w2 = [&](int x, int y) {
          const int kk = p2(i2, m, x, y);
          return nA * B2[kk] - nB * A2[kk];
        };
        A3[q] = A3[q] + B3[q] + nA * nB * (nA - nB) / (n * n) * d(a) * d(b) * d(c) +
                (d(a) * w2(b, c) + d(b) * w2(a, c) + d(c) * w2(a, b)) / n;
      }
      __syncthreads();
      for (int q = t; q < sh.P2; q += kMomThreads) {
        const uint32_t cd = T.code[m + q];
        const int a = cidx(cd, 0), b = cidx(cd, 1);
        A2[q] = A2[q] + B2[q] + nA * nB / n * d(a) * d(b);
      }
      if (t < m) A1[t] = A1[t] + d(t) * (nB / n);
      nAi += nBi;
      __syncthreads();
    }
    if (t == 0) out.n[j] = nAi;
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
  auto code = a.template take<uint32_t>(sh.U);
  auto idx2 = a.template take<uint16_t>((size_t)sh.m * sh.m);
  auto idx3 = a.template take<uint16_t>((size_t)sh.m * sh.m * sh.m);
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
  const unsigned grid1 = (unsigned)std::min<int64_t>((int64_t)J, 65535);
  if (J)
    hipLaunchKernelGGL(k_mom_merge, dim3(grid1), dim3(kMomThreads), 0, s, J, W.job_lo, W.job_hi, in, W.part, sh,
                       W.tab);
  // second level: the chunk results of every group, in order
  MergeIn in2;
  in2.n = W.part.n;
  in2.mean = W.part.mean;
  in2.m2 = W.part.m2;
  in2.m3 = W.part.m3;
  in2.m4 = W.part.m4;
  in2.map = nullptr;
  const unsigned grid2 = (unsigned)std::min<int64_t>((int64_t)G, 65535);
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
    const unsigned passes = (unsigned)((sh.U + kMomChunk - 1) / kMomChunk);
    hipLaunchKernelGGL(k_mom_cells, dim3((unsigned)std::min<uint32_t>(S, 65535), passes), dim3(kMomThreads), 0, s,
                       W.perm, W.lay.cell_off, W.lay.order, d_sites, S, d_vars, g.n, sh, W.tab, co);
    hipLaunchKernelGGL(k_mom_center, dim3((unsigned)std::min<uint32_t>(S, 65535)), dim3(kMomThreads), 0, s,
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
