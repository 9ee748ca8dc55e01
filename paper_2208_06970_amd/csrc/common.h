// Internal helpers shared by the gfx950 kernels and the C ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/lsrvt.h"

namespace lsrvt {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint64_t kInfKey = 0xFFFFFFFFFFFFFFFFull;
constexpr int kWave = 64;

struct Geom {
  int32_t nx, ny, nz;
  int64_t n;
};

// Validate dims against the library limits; fills g.
inline int32_t make_geom(lsrvt_dims d, Geom &g) {
  if (d.nx <= 0 || d.ny <= 0 || d.nz <= 0) return LSRVT_EINVAL;
  if (d.nx > 32767 || d.ny > 32767 || d.nz > 32767) return LSRVT_ELIMIT;
  int64_t n = (int64_t)d.nx * d.ny * d.nz;
  if (n > 2147483647LL) return LSRVT_ELIMIT;
  g.nx = d.nx;
  g.ny = d.ny;
  g.nz = d.nz;
  g.n = n;
  return LSRVT_OK;
}

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

#define LSRVT_HIP(call)                                  \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return LSRVT_EDEVICE;          \
  } while (0)

#define LSRVT_LAUNCHED()                                  \
  do {                                                    \
    hipError_t e_ = hipGetLastError();                    \
    if (e_ != hipSuccess) return LSRVT_EDEVICE;           \
  } while (0)

// Bump allocator over the caller's workspace; every slice is 256-byte aligned.
struct Carve {
  uint8_t *base;
  size_t size;
  size_t off = 0;
  bool ok = true;
  Carve(void *b, size_t s) : base(static_cast<uint8_t *>(b)), size(s) {}
  template <class T>
  T *take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    if (off + bytes > size) {
      ok = false;
      return nullptr;
    }
    T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
    off += bytes;
    return p;
  }
};

// Same layout walk with no buffer: used by the *_workspace queries.
struct Sizer {
  size_t off = 0;
  template <class T>
  T *take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    off += bytes;
    return nullptr;
  }
};

inline int32_t check_work(void *d_work, size_t have, size_t need) {
  if (need == 0) return LSRVT_OK;
  if (!d_work || have < need || (reinterpret_cast<uintptr_t>(d_work) & 255u)) return LSRVT_EWORKSPACE;
  return LSRVT_OK;
}

inline unsigned grid_for(int64_t items, int per_block, int64_t cap = 1 << 20) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// ---------------------------------------------------------------------------
// device helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Float <-> order-preserving uint32 key (for exact atomic min/max of floats).
__device__ __forceinline__ uint32_t f2key(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ __forceinline__ float key2f(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
#if defined(__HIP_DEVICE_COMPILE__)
  return __uint_as_float(u);
#else
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
#endif
}

// Wave-wide sum of a 64-bit value (all 64 lanes must participate).
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Slot of key c in an open-addressing LDS table of Cap keys (kNone = empty),
// inserting it if absent; -1 when the table is full.
template <int Cap>
__device__ __forceinline__ int lds_slot(uint32_t *keys, uint32_t c) {
  uint32_t h = (c * 2654435761u) & (Cap - 1);
  for (int probe = 0; probe < Cap; ++probe) {
    uint32_t k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (k == c) return (int)h;
    if (k == kNone) {
      uint32_t old = atomicCAS(&keys[h], kNone, c);
      if (old == kNone || old == c) return (int)h;
    }
    h = (h + 1) & (Cap - 1);
  }
  return -1;
}

// Fill kernel used instead of hipMemsetAsync (graph-capture safe).
template <class T>
__global__ void k_fill(T *p, int64_t n, T v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

template <class T>
inline int32_t fill(T *p, int64_t n, T v, hipStream_t s) {
  if (n <= 0) return LSRVT_OK;
  hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
  LSRVT_LAUNCHED();
  return LSRVT_OK;
}

// The Lloyd loops of many jobs in lockstep, one launch per phase over all
// jobs (cvt.hip); used by lsrvt_batch_run.
struct CvtBatchJob {
  lsrvt_dims dims;
  const uint8_t *band;
  const uint32_t *comp;
  const uint32_t *seeds;
  uint32_t n_sites;
  const uint16_t *weights;
  int32_t iters;
  uint32_t *cell, *sites, *site_comp;
};
// Launch-shape settings of the calling host thread (lsrvt_set_tuning); 0 =
// the library's choice.
int32_t tuning(int32_t knob);

size_t cvt_batch_header(int32_t n);
size_t cvt_batch_job_workspace(lsrvt_dims dims, uint32_t n_sites, int32_t iters);
int32_t cvt_batch(const CvtBatchJob *jobs, int32_t n, void *work, size_t bytes, int32_t *status, hipStream_t s);

// Reads n <= 64 words of device memory to the host after the work queued on
// s (synchronises s).  Implemented in readback.hip.
int32_t read_words(const uint32_t *d_src, int n, uint32_t *h_out, hipStream_t s);

// ---------------------------------------------------------------------------
// Stable counting sort of a u32 index list by an 8-bit key, used for the
// band ordering of component roots and (per digit) for sorting sites by
// component.  Implemented in sort.hip.
struct StableSort8 {
  static size_t workspace(int64_t n);
  // keys[i] (8-bit digit of element i) -> out_pos[i] = destination of i.
  // If bucket_offset is non-null it receives the 257 exclusive bucket starts.
  static int32_t run(const uint8_t *keys, int64_t n, uint32_t *out_pos, uint32_t *bucket_offset,
                     void *work, size_t work_bytes, hipStream_t s);
};

// Exclusive scan of uint32 counts (n <= 2^31) into offsets[n+1]; device-wide.
struct ScanU32 {
  static size_t workspace(int64_t n);
  static int32_t run(const uint32_t *in, int64_t n, uint32_t *out, void *work, size_t work_bytes,
                     hipStream_t s);
};

}  // namespace lsrvt
