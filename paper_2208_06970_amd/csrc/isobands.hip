// Isoband classification (Sec. 3.1, B_{a,b} = { v : a < f(v) <= b }).
//
// One streaming pass: 4 B read + 1 B written per voxel.  Each thread
// classifies 16 consecutive voxels (four float4 loads, one 16-byte store).
// The isovalues arrive as a kernel argument (they sit in scalar registers);
// the band is the branch-free count of isovalues strictly below the value.
// Large isovalue counts use a binary search over a copy in LDS instead.
#include "common.h"

namespace lsrvt {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct IsoArg {
  float v[256];
};

constexpr int kIsoThreads = 256;
constexpr int kIsoVec = 16;

template <int K>
__device__ __forceinline__ uint32_t count_below_fixed(float x, const IsoArg &iso) {
  uint32_t b = 0;
#pragma unroll
  for (int i = 0; i < K; ++i) b += (iso.v[i] < x) ? 1u : 0u;
  return b;
}

__device__ __forceinline__ uint32_t count_below_search(float x, const float *lds_iso, int k) {
  // smallest i with !(iso[i] < x), i.e. #{iso < x}; NaN compares false -> 0
  int lo = 0, hi = k;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (lds_iso[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (uint32_t)lo;
}

template <int K>
__global__ __launch_bounds__(kIsoThreads) void k_isobands(const float *__restrict__ f, int64_t n, IsoArg iso, int k,
                                                          uint8_t *__restrict__ band, uint32_t *status) {
  __shared__ float lds_iso[256];
  if (K < 0) {
    for (int i = threadIdx.x; i < k; i += kIsoThreads) lds_iso[i] = iso.v[i];
    __syncthreads();
  }
  auto classify = [&](float x) -> uint32_t {
    if constexpr (K >= 0)
      return count_below_fixed<K>(x, iso);
    else
      return count_below_search(x, lds_iso, k);
  };
  bool nan = false;
  const int64_t nvec = n / kIsoVec;
  const bool aligned = ((reinterpret_cast<uintptr_t>(f) & 15u) == 0) && ((reinterpret_cast<uintptr_t>(band) & 15u) == 0);
  int64_t t = (int64_t)blockIdx.x * kIsoThreads + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kIsoThreads;
  if (aligned) {
    for (int64_t i = t; i < nvec; i += stride) {
      const f32x4 *src = reinterpret_cast<const f32x4 *>(f + i * kIsoVec);
      f32x4 a = __builtin_nontemporal_load(src + 0);
      f32x4 b = __builtin_nontemporal_load(src + 1);
      f32x4 c = __builtin_nontemporal_load(src + 2);
      f32x4 d = __builtin_nontemporal_load(src + 3);
      float xs[16] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3], c[0], c[1], c[2], c[3], d[0], d[1], d[2], d[3]};
      uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        nan |= (xs[j] != xs[j]);
        w[j >> 2] |= classify(xs[j]) << (8 * (j & 3));
      }
      uint4 o;
      o.x = w[0];
      o.y = w[1];
      o.z = w[2];
      o.w = w[3];
      *reinterpret_cast<uint4 *>(band + i * kIsoVec) = o;
    }
  }
  const int64_t tail0 = aligned ? nvec * kIsoVec : 0;
  for (int64_t i = tail0 + t; i < n; i += stride) {
    float x = f[i];
    nan |= (x != x);
    band[i] = (uint8_t)classify(x);
  }
  uint64_t any = __ballot(nan);
  if (status && any && lane_id() == 0) atomicOr(status, 1u);
}

template <int K>
void launch(const float *f, int64_t n, const IsoArg &iso, int k, uint8_t *band, uint32_t *status, hipStream_t s) {
  int64_t work = (n + kIsoVec - 1) / kIsoVec;
  unsigned g = grid_for(work, kIsoThreads, 1 << 16);
  hipLaunchKernelGGL(k_isobands<K>, dim3(g), dim3(kIsoThreads), 0, s, f, n, iso, k, band, status);
}

}  // namespace

}  // namespace lsrvt

using namespace lsrvt;

extern "C" int32_t lsrvt_isobands(const float *d_field, lsrvt_dims dims, const float *h_iso, int32_t n_iso,
                                  uint8_t *d_band, uint32_t *d_status, void *stream) {
  Geom g;
  int32_t st = make_geom(dims, g);
  if (st) return st;
  if (!d_field || !d_band) return LSRVT_EINVAL;
  if (n_iso < 0 || n_iso > 254) return LSRVT_EINVAL;
  if (n_iso > 0 && !h_iso) return LSRVT_EINVAL;
  IsoArg iso;
  for (int i = 0; i < 256; ++i) iso.v[i] = 0.0f;
  for (int32_t i = 0; i < n_iso; ++i) {
    float v = h_iso[i];
    if (!(v == v) || v == __builtin_inff() || v == -__builtin_inff()) return LSRVT_EINVAL;
    if (i > 0 && !(h_iso[i - 1] < v)) return LSRVT_EINVAL;
    iso.v[i] = v;
  }
  hipStream_t s = as_stream(stream);
  if (d_status) {
    st = fill<uint32_t>(d_status, 1, 0u, s);
    if (st) return st;
  }
  switch (n_iso) {
#define LSRVT_ISO_CASE(K) \
  case K:                 \
    launch<K>(d_field, g.n, iso, n_iso, d_band, d_status, s); \
    break;
    LSRVT_ISO_CASE(0)
    LSRVT_ISO_CASE(1)
    LSRVT_ISO_CASE(2)
    LSRVT_ISO_CASE(3)
    LSRVT_ISO_CASE(4)
    LSRVT_ISO_CASE(5)
    LSRVT_ISO_CASE(6)
    LSRVT_ISO_CASE(7)
    LSRVT_ISO_CASE(8)
    LSRVT_ISO_CASE(9)
    LSRVT_ISO_CASE(10)
    LSRVT_ISO_CASE(11)
    LSRVT_ISO_CASE(12)
    LSRVT_ISO_CASE(13)
    LSRVT_ISO_CASE(14)
    LSRVT_ISO_CASE(15)
    LSRVT_ISO_CASE(16)
#undef LSRVT_ISO_CASE
    default:
      launch<-1>(d_field, g.n, iso, n_iso, d_band, d_status, s);
  }
  LSRVT_LAUNCHED();
  return LSRVT_OK;
}
