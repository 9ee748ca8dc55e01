// Device-wide exclusive scan of uint32 counts and a stable counting sort by
// an 8-bit key.  Both are deterministic: results do not depend on scheduling.
#include "common.h"

namespace lsrvt {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

// Inclusive scan of one value per thread across a 256-thread block.
__device__ uint32_t block_inclusive_scan(uint32_t v, uint32_t *lds_waves /*[4]*/, uint32_t &total) {
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t t = __shfl_up(v, o, kWave);
    if (lane >= o) v += t;
  }
  if (lane == kWave - 1) lds_waves[wid] = v;
  __syncthreads();
  uint32_t add = 0;
  for (int w = 0; w < wid; ++w) add += lds_waves[w];
  total = lds_waves[0] + lds_waves[1] + lds_waves[2] + lds_waves[3];
  __syncthreads();
  return v + add;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t *in, int64_t n, uint32_t *block_sums) {
  __shared__ uint32_t lw[4];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += in[base + i];
  uint32_t total;
  block_inclusive_scan(s, lw, total);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Single-block exclusive scan of the per-tile sums (any length), in place.
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(uint32_t *sums, int64_t nb) {
  __shared__ uint32_t lw[4];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += kScanThreads) {
    int64_t i = base + threadIdx.x;
    uint32_t v = i < nb ? sums[i] : 0u;
    uint32_t total;
    uint32_t inc = block_inclusive_scan(v, lw, total);
    uint32_t c = carry;
    if (i < nb) sums[i] = c + inc - v;
    __syncthreads();
    if (threadIdx.x == 0) carry = c + total;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t *in, int64_t n, const uint32_t *tile_off,
                                                              uint32_t *out) {
  __shared__ uint32_t lw[4];
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : 0u;
    s += v[i];
  }
  uint32_t total;
  uint32_t inc = block_inclusive_scan(s, lw, total);
  uint32_t run = tile_off[blockIdx.x] + inc - s;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
    if (base + i == n - 1) out[n] = run;
  }
}

constexpr int kSortChunk = 1024;  // elements per wave in the stable sort

// Per-chunk histograms of the 8-bit keys, stored key-major: hist[key * nch + chunk].
__global__ __launch_bounds__(kWave) void k_sort8_hist(const uint8_t *keys, int64_t n, int64_t nch, uint32_t *hist) {
  __shared__ uint32_t h[256];
  for (int i = threadIdx.x; i < 256; i += kWave) h[i] = 0;
  __syncthreads();
  int64_t c = blockIdx.x;
  int64_t base = c * kSortChunk;
  for (int i = threadIdx.x; i < kSortChunk; i += kWave) {
    int64_t e = base + i;
    if (e < n) atomicAdd(&h[keys[e]], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += kWave) hist[(int64_t)i * nch + c] = h[i];
}

// Stable scatter: one wave walks its chunk in order, 64 elements at a time;
// equal keys inside a group are ranked by lane with ballots over the 8 key bits.
__global__ __launch_bounds__(kWave) void k_sort8_scatter(const uint8_t *keys, int64_t n, int64_t nch,
                                                          const uint32_t *off, uint32_t *out_pos) {
  __shared__ uint32_t run[256];
  int64_t c = blockIdx.x;
  for (int i = threadIdx.x; i < 256; i += kWave) run[i] = off[(int64_t)i * nch + c];
  __syncthreads();
  int64_t base = c * kSortChunk;
  for (int g = 0; g < kSortChunk; g += kWave) {
    int64_t e = base + g + threadIdx.x;
    bool valid = e < n;
    uint32_t k = valid ? keys[e] : 0u;
    uint64_t vmask = __ballot(valid);
    uint64_t same = vmask;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t bal = __ballot((k >> b) & 1u);
      same &= ((k >> b) & 1u) ? bal : ~bal;
    }
    uint32_t pos = 0;
    if (valid) pos = run[k] + (uint32_t)__popcll(same & lanemask_lt());
    __syncthreads();
    if (valid) {
      out_pos[e] = pos;
      // the highest lane of each equal-key group advances the running offset
      if ((same >> threadIdx.x) == 1ull) run[k] += (uint32_t)__popcll(same);
    }
    __syncthreads();
  }
}

__global__ void k_sort8_buckets(const uint32_t *off, int64_t nch, int64_t n, uint32_t *bucket_offset) {
  int i = threadIdx.x;
  if (i < 256) bucket_offset[i] = off[(int64_t)i * nch];
  if (i == 0) bucket_offset[256] = (uint32_t)n;
}

}  // namespace

size_t ScanU32::workspace(int64_t n) {
  Sizer z;
  z.take<uint32_t>((n + kScanTile - 1) / kScanTile + 1);
  return z.off;
}

int32_t ScanU32::run(const uint32_t *in, int64_t n, uint32_t *out, void *work, size_t work_bytes, hipStream_t s) {
  if (n <= 0) {
    return fill<uint32_t>(out, 1, 0u, s);
  }
  Carve cv(work, work_bytes);
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  uint32_t *sums = cv.take<uint32_t>(nb + 1);
  if (!cv.ok) return LSRVT_EWORKSPACE;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, sums);
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanThreads), 0, s, sums, nb);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, sums, out);
  LSRVT_LAUNCHED();
  return LSRVT_OK;
}

size_t StableSort8::workspace(int64_t n) {
  int64_t nch = (n + kSortChunk - 1) / kSortChunk;
  if (nch < 1) nch = 1;
  Sizer z;
  z.take<uint32_t>(256 * nch);
  z.take<uint32_t>(256 * nch + 1);
  z.off += ScanU32::workspace(256 * nch);
  return z.off;
}

int32_t StableSort8::run(const uint8_t *keys, int64_t n, uint32_t *out_pos, uint32_t *bucket_offset, void *work,
                         size_t work_bytes, hipStream_t s) {
  int64_t nch = (n + kSortChunk - 1) / kSortChunk;
  if (nch < 1) nch = 1;
  Carve cv(work, work_bytes);
  uint32_t *hist = cv.take<uint32_t>(256 * nch);
  uint32_t *off = cv.take<uint32_t>(256 * nch + 1);
  if (!cv.ok) return LSRVT_EWORKSPACE;
  void *rest = cv.base + cv.off;
  size_t rest_bytes = cv.size - cv.off;
  hipLaunchKernelGGL(k_sort8_hist, dim3((unsigned)nch), dim3(kWave), 0, s, keys, n, nch, hist);
  LSRVT_LAUNCHED();
  int32_t st = ScanU32::run(hist, 256 * nch, off, rest, rest_bytes, s);
  if (st) return st;
  if (n > 0) {
    hipLaunchKernelGGL(k_sort8_scatter, dim3((unsigned)nch), dim3(kWave), 0, s, keys, n, nch, off, out_pos);
    LSRVT_LAUNCHED();
  }
  if (bucket_offset) {
    hipLaunchKernelGGL(k_sort8_buckets, dim3(1), dim3(256), 0, s, off, nch, n, bucket_offset);
    LSRVT_LAUNCHED();
  }
  return LSRVT_OK;
}

}  // namespace lsrvt
