// Many independent jobs (volumes) through the whole path in one call: each
// job runs isobands -> components -> Lloyd loop -> statistics, exactly as the
// four single-job calls would, on one of several HIP streams, so that small
// jobs overlap on the GPU and the host waits of one job (component count,
// level checks) do not stall the others.  Each stream has its own slice of
// the caller's workspace, sized for the largest job, and a host thread that
// takes the next job when its previous job has been enqueued.  Every job's
// results are bit-identical to running it alone: the kernels and their
// reduction orders do not depend on what else runs on the device.
#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

#include "common.h"

namespace lsrvt {
namespace {

size_t job_workspace(const lsrvt_job &j) {
  const int32_t nb = j.n_iso + 1;
  size_t a = lsrvt_components_workspace(j.dims, nb);
  size_t b = lsrvt_cvt_workspace(j.dims, j.n_sites, j.iters < 0 ? 0 : j.iters);
  size_t c = lsrvt_aggregate_workspace(j.dims, j.n_sites, j.cap_comp, nb, j.n_vars, j.n_bins, j.flags);
  if (a == 0 || b == 0 || c == 0) return 0;
  size_t m = std::max(a, std::max(b, c));
  return (m + 255) & ~size_t(255);
}

int32_t run_job(lsrvt_job &j, void *work, size_t bytes, hipStream_t s) {
  const int32_t nb = j.n_iso + 1;
  int32_t rc = lsrvt_isobands(j.d_field, j.dims, j.h_iso, j.n_iso, j.d_band, j.d_status, s);
  if (rc) return rc;
  uint32_t n_comp = 0;
  rc = lsrvt_components(j.d_band, j.dims, nb, j.d_comp, j.cap_comp, j.d_comp_band, j.d_comp_size, j.d_comp_first,
                        j.d_band_offset, &n_comp, work, bytes, s);
  j.n_comp = n_comp;
  if (rc) return rc;
  rc = lsrvt_cvt(j.d_band, j.d_comp, j.dims, j.d_seeds, j.n_sites, j.d_weights, j.iters, j.d_cell, j.d_sites,
                 j.d_site_comp, nullptr, work, bytes, s);
  if (rc) return rc;
  rc = lsrvt_aggregate(j.d_cell, j.dims, j.d_sites, j.d_site_comp, j.n_sites, j.d_comp_band, n_comp, nb, j.d_vars,
                       j.n_vars, j.d_edges, j.n_bins, j.flags, &j.cell, &j.comp, &j.band, work, bytes, s);
  if (rc) return rc;
  LSRVT_HIP(hipStreamSynchronize(s));
  return LSRVT_OK;
}

}  // namespace
}  // namespace lsrvt

using namespace lsrvt;

extern "C" size_t lsrvt_batch_workspace(const lsrvt_job *jobs, int32_t n_jobs, int32_t n_streams) {
  if (!jobs || n_jobs < 0 || n_streams < 1) return 0;
  size_t m = 256;
  for (int32_t i = 0; i < n_jobs; ++i) {
    const size_t w = job_workspace(jobs[i]);
    if (w == 0) return 0;
    m = std::max(m, w);
  }
  const int32_t slots = std::min<int32_t>(n_streams, std::max<int32_t>(n_jobs, 1));
  return m * (size_t)slots;
}

extern "C" int32_t lsrvt_batch_run(lsrvt_job *jobs, int32_t n_jobs, int32_t n_streams, void *d_work,
                                   size_t work_bytes, void *stream) {
  if (n_jobs < 0 || n_streams < 1 || (n_jobs > 0 && !jobs)) return LSRVT_EINVAL;
  if (n_jobs == 0) return LSRVT_OK;
  for (int32_t i = 0; i < n_jobs; ++i) {
    jobs[i].status = LSRVT_EINVAL;
    jobs[i].n_comp = 0;
    if (job_workspace(jobs[i]) == 0) return LSRVT_EINVAL;
  }
  size_t per = 256;
  for (int32_t i = 0; i < n_jobs; ++i) per = std::max(per, job_workspace(jobs[i]));
  const int32_t slots = std::min(n_streams, n_jobs);
  int32_t rc = check_work(d_work, work_bytes, per * (size_t)slots);
  if (rc) return rc;
  int dev = 0;
  LSRVT_HIP(hipGetDevice(&dev));
  hipStream_t caller = as_stream(stream);
  // the jobs' inputs are ready once the caller's stream reaches this point
  hipEvent_t ready;
  LSRVT_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  if (hipEventRecord(ready, caller) != hipSuccess) {
    hipEventDestroy(ready);
    return LSRVT_EDEVICE;
  }
  std::atomic<int32_t> next{0};
  std::atomic<int32_t> failed{0};
  std::vector<std::thread> pool;
  pool.reserve(slots);
  for (int32_t k = 0; k < slots; ++k) {
    pool.emplace_back([&, k]() {
      if (hipSetDevice(dev) != hipSuccess) {
        failed.store(1);
        return;
      }
      hipStream_t s;
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        failed.store(1);
        return;
      }
      if (hipStreamWaitEvent(s, ready, 0) != hipSuccess) failed.store(1);
      void *work = static_cast<uint8_t *>(d_work) + per * (size_t)k;
      while (!failed.load()) {
        const int32_t i = next.fetch_add(1);
        if (i >= n_jobs) break;
        jobs[i].status = run_job(jobs[i], work, per, s);
      }
      hipStreamSynchronize(s);
      hipStreamDestroy(s);
    });
  }
  for (auto &th : pool) th.join();
  hipEventDestroy(ready);
  if (failed.load()) return LSRVT_EDEVICE;
  for (int32_t i = 0; i < n_jobs; ++i)
    if (jobs[i].status != LSRVT_OK) return jobs[i].status;
  return LSRVT_OK;
}
