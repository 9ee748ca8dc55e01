// Small device-to-host reads on the host's control path (flags, counts,
// sizes that decide the next launches).  A copy kernel writes the words into
// pinned, device-mapped host memory and the host reads them after the
// stream synchronises: a few microseconds instead of a staged runtime copy.
// Buffers come from a process-wide pool (one per concurrent reader) and are
// kept until the process ends.
#include <mutex>
#include <vector>

#include "common.h"

namespace lsrvt {

namespace {

constexpr int kReadWords = 64;

struct PinnedBuf {
  uint32_t *host = nullptr;
  uint32_t *dev = nullptr;
};

struct PinnedPool {
  std::mutex mu;
  std::vector<PinnedBuf> free;
};

PinnedPool &pool() {
  static PinnedPool p;
  return p;
}

__global__ void k_read_words(const uint32_t *__restrict__ src, int n, uint32_t *dst) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace

int32_t read_words(const uint32_t *d_src, int n, uint32_t *h_out, hipStream_t s) {
  if (n <= 0) return LSRVT_OK;
  if (n > kReadWords) return LSRVT_EINVAL;
  PinnedBuf b;
  {
    std::lock_guard<std::mutex> lk(pool().mu);
    if (!pool().free.empty()) {
      b = pool().free.back();
      pool().free.pop_back();
    }
  }
  if (!b.host) {
    void *h = nullptr;
    LSRVT_HIP(hipHostMalloc(&h, kReadWords * sizeof(uint32_t), hipHostMallocMapped | hipHostMallocCoherent));
    void *d = nullptr;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess || !d) {
      (void)hipHostFree(h);
      return LSRVT_EDEVICE;
    }
    b.host = static_cast<uint32_t *>(h);
    b.dev = static_cast<uint32_t *>(d);
  }
  int32_t rc = LSRVT_OK;
  hipLaunchKernelGGL(k_read_words, dim3(1), dim3(kReadWords), 0, s, d_src, n, b.dev);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    rc = LSRVT_EDEVICE;
  } else {
    for (int i = 0; i < n; ++i) h_out[i] = __atomic_load_n(&b.host[i], __ATOMIC_ACQUIRE);
  }
  std::lock_guard<std::mutex> lk(pool().mu);
  pool().free.push_back(b);
  return rc;
}

}  // namespace lsrvt
