// Many independent jobs (volumes) through the whole path in one call, in
// three phases:
//  1. isobands and components of every job, on several HIP streams driven by
//     host threads (each stream with its own slice of the workspace), so small
//     jobs overlap and one job's host wait (its component count) does not stall
//     the others;
//  2. the Lloyd loops of all jobs in lockstep: every phase of every pass is
//     one launch over all jobs (cvt.hip, cvt_batch), the Voronoi passes by the
//     brick relaxation, with relaxation rounds shared by the jobs;
//  3. the statistics of every job, on the streams again.
// Every job's results are bit-identical to running its four calls alone: the
// kernels and their reduction orders are the job's own, and both schedules of
// the Voronoi passes reach the same regions.
#include <algorithm>
#include <atomic>
#include <functional>
#include <thread>
#include <vector>

#include "common.h"

namespace lsrvt {
namespace {

size_t slice_workspace(const lsrvt_job &j) {
  const int32_t nb = j.n_iso + 1;
  size_t a = lsrvt_components_workspace(j.dims, nb);
  size_t c = lsrvt_aggregate_workspace(j.dims, j.n_sites, j.cap_comp, nb, j.n_vars, j.n_bins, j.flags);
  if (a == 0 || c == 0) return 0;
  return (std::max(a, c) + 255) & ~size_t(255);
}

size_t lloyd_workspace(const lsrvt_job *jobs, int32_t n) {
  size_t total = cvt_batch_header(n);
  for (int32_t i = 0; i < n; ++i) {
    const size_t w = cvt_batch_job_workspace(jobs[i].dims, jobs[i].n_sites, jobs[i].iters < 0 ? 0 : jobs[i].iters);
    if (w == 0) return 0;
    total += w;
  }
  return total;
}

int32_t labels(lsrvt_job &j, void *work, size_t bytes, hipStream_t s) {
  const int32_t nb = j.n_iso + 1;
  int32_t rc = lsrvt_isobands(j.d_field, j.dims, j.h_iso, j.n_iso, j.d_band, j.d_status, s);
  if (rc) return rc;
  uint32_t n_comp = 0;
  rc = lsrvt_components(j.d_band, j.dims, nb, j.d_comp, j.cap_comp, j.d_comp_band, j.d_comp_size, j.d_comp_first,
                        j.d_band_offset, &n_comp, work, bytes, s);
  j.n_comp = n_comp;
  return rc;
}

int32_t statistics(lsrvt_job &j, void *work, size_t bytes, hipStream_t s) {
  const int32_t nb = j.n_iso + 1;
  int32_t rc = lsrvt_aggregate(j.d_cell, j.dims, j.d_sites, j.d_site_comp, j.n_sites, j.d_comp_band, j.n_comp, nb,
                               j.d_vars, j.n_vars, j.d_edges, j.n_bins, j.flags, &j.cell, &j.comp, &j.band, work,
                               bytes, s);
  if (rc) return rc;
  LSRVT_HIP(hipStreamSynchronize(s));
  return LSRVT_OK;
}

// Runs fn(job, slice, bytes, stream) for every job whose status is still OK,
// on `slots` streams (host threads) that first wait for `ready`.
int32_t on_streams(lsrvt_job *jobs, int32_t n, int32_t slots, uint8_t *work, size_t per, hipEvent_t ready, int dev,
                   const std::function<int32_t(lsrvt_job &, void *, size_t, hipStream_t)> &fn) {
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
      void *slice = work + per * (size_t)k;
      while (!failed.load()) {
        const int32_t i = next.fetch_add(1);
        if (i >= n) break;
        if (jobs[i].status == LSRVT_OK) jobs[i].status = fn(jobs[i], slice, per, s);
      }
      if (hipStreamSynchronize(s) != hipSuccess) failed.store(1);
      (void)hipStreamDestroy(s);
    });
  }
  for (auto &th : pool) th.join();
  return failed.load() ? LSRVT_EDEVICE : LSRVT_OK;
}

}  // namespace
}  // namespace lsrvt

using namespace lsrvt;

extern "C" size_t lsrvt_batch_workspace(const lsrvt_job *jobs, int32_t n_jobs, int32_t n_streams) {
  if (!jobs || n_jobs < 0 || n_streams < 1) return 0;
  size_t m = 256;
  for (int32_t i = 0; i < n_jobs; ++i) {
    const size_t w = slice_workspace(jobs[i]);
    if (w == 0) return 0;
    m = std::max(m, w);
  }
  const int32_t slots = std::min<int32_t>(n_streams, std::max<int32_t>(n_jobs, 1));
  const size_t lloyd = lloyd_workspace(jobs, n_jobs);
  if (lloyd == 0) return 0;
  return std::max(m * (size_t)slots, lloyd);
}

extern "C" int32_t lsrvt_batch_run(lsrvt_job *jobs, int32_t n_jobs, int32_t n_streams, void *d_work,
                                   size_t work_bytes, void *stream) {
  if (n_jobs < 0 || n_streams < 1 || (n_jobs > 0 && !jobs)) return LSRVT_EINVAL;
  if (n_jobs == 0) return LSRVT_OK;
  for (int32_t i = 0; i < n_jobs; ++i) {
    jobs[i].status = LSRVT_EINVAL;
    jobs[i].n_comp = 0;
    if (slice_workspace(jobs[i]) == 0 || jobs[i].iters < 0) return LSRVT_EINVAL;
  }
  size_t per = 256;
  for (int32_t i = 0; i < n_jobs; ++i) per = std::max(per, slice_workspace(jobs[i]));
  const int32_t slots = std::min(n_streams, n_jobs);
  int32_t rc = check_work(d_work, work_bytes, lsrvt_batch_workspace(jobs, n_jobs, n_streams));
  if (rc) return rc;
  for (int32_t i = 0; i < n_jobs; ++i) jobs[i].status = LSRVT_OK;
  int dev = 0;
  LSRVT_HIP(hipGetDevice(&dev));
  hipStream_t caller = as_stream(stream);
  uint8_t *work = static_cast<uint8_t *>(d_work);
  // the jobs' inputs are ready once the caller's stream reaches this point
  hipEvent_t ready;
  LSRVT_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  if (hipEventRecord(ready, caller) != hipSuccess) {
    (void)hipEventDestroy(ready);
    return LSRVT_EDEVICE;
  }
  // 1. labels of every job
  rc = on_streams(jobs, n_jobs, slots, work, per, ready, dev, labels);
  if (rc == LSRVT_OK) {
    // 2. the Lloyd loops in lockstep, over the jobs whose labels succeeded
    std::vector<CvtBatchJob> cj;
    std::vector<int32_t> idx, st;
    for (int32_t i = 0; i < n_jobs; ++i) {
      if (jobs[i].status != LSRVT_OK) continue;
      const lsrvt_job &j = jobs[i];
      cj.push_back(CvtBatchJob{j.dims, j.d_band, j.d_comp, j.d_seeds, j.n_sites, j.d_weights, j.iters, j.d_cell,
                               j.d_sites, j.d_site_comp});
      idx.push_back(i);
    }
    st.assign(cj.size(), LSRVT_OK);
    const int32_t crc = cvt_batch(cj.data(), (int32_t)cj.size(), work, work_bytes, st.data(), caller);
    for (size_t k = 0; k < idx.size(); ++k) jobs[idx[k]].status = crc ? crc : st[k];
    // 3. statistics of every job
    if (hipEventRecord(ready, caller) != hipSuccess) rc = LSRVT_EDEVICE;
    if (rc == LSRVT_OK) rc = on_streams(jobs, n_jobs, slots, work, per, ready, dev, statistics);
  }
  if (hipStreamSynchronize(caller) != hipSuccess && rc == LSRVT_OK) rc = LSRVT_EDEVICE;
  (void)hipEventDestroy(ready);
  if (rc) return rc;
  for (int32_t i = 0; i < n_jobs; ++i)
    if (jobs[i].status != LSRVT_OK) return jobs[i].status;
  return LSRVT_OK;
}
