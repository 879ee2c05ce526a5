// noalloc.hip -- a job list run without any allocation, for callers that
// cannot allocate device memory (code under stream capture, tight serving
// loops).
//
// raid6c_run_jobs_noalloc runs the same work as a plan's grouped schedule
// (one grid of each prime's job-list kernel), but instead of tables that a
// plan allocates and keeps, the job and item tables are staged, on every
// call, in `scratch`: a fixed array in device memory that each GPU the
// library runs on holds until the process ends.  The tables are built in a
// fixed host array and copied from it; the runtime performs a copy from
// pageable host memory synchronously, so the host array is free again when
// the copy call returns, and the copy waits for the work queued before it on
// the same stream (an earlier call's kernels, which read the tables).
#include <hip/hip_runtime.h>

#include <string.h>

#include <mutex>

#include "../../include/raid6c.h"
#include "raid6c_internal.h"

namespace raid6c {

int fail(int code, const char* fmt, ...);

namespace {

constexpr size_t kNoAllocJobs = RAID6C_NOALLOC_MAX_JOBS;
constexpr size_t kNoAllocItems = RAID6C_NOALLOC_MAX_ITEMS;
constexpr size_t kJobsBytes = (kNoAllocJobs * sizeof(BatchJob) + 255) / 256 * 256;
constexpr size_t kScratchBytes = kJobsBytes + kNoAllocItems * sizeof(BatchItem);
constexpr int kMaxDevices = 64;

// The device tables: jobs, then items.  In host code the name stands for a
// host-side handle, not a device address; the address comes from
// hipGetSymbolAddress (per device) and only that is passed on.
__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_mu;                           // guards everything below
uint8_t* g_scratch[kMaxDevices] = {};      // scratch's address on each device
BatchJob g_jobs[kNoAllocJobs];             // host staging of the tables
BatchItem g_items[kNoAllocItems];

int scratch_on(int dev, uint8_t** out) {
  if (g_scratch[dev] == nullptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      return fail(RAID6C_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch[dev] = (uint8_t*)ptr;
  }
  *out = g_scratch[dev];
  return RAID6C_OK;
}

}  // namespace
}  // namespace raid6c

using namespace raid6c;

extern "C" int raid6c_run_jobs_noalloc(const raid6c_job* jobs, size_t njobs, void* stream) {
  if (jobs == nullptr && njobs != 0) return fail(RAID6C_E_ARG, "jobs is NULL");
  if (njobs > kNoAllocJobs)
    return fail(RAID6C_E_ARG, "%zu jobs: at most %zu without allocation", njobs, kNoAllocJobs);
  // Checks, and the items of each group (prime, and plain or extended Q
  // parity): tiles of 64 lanes x that prime's job-list vector width, jobs in
  // the order given.
  size_t per_group[2][kMaxPrime + 1] = {};
  size_t nitems = 0;
  for (size_t i = 0; i < njobs; ++i) {
    Case cs;
    const int rc = check_job(jobs[i], i, &cs);
    if (rc != RAID6C_OK) return rc;
    const uint32_t tile = 64u * 4u * (uint32_t)zp_prime_entry(jobs[i].p)->group_vec;
    const size_t n = (jobs[i].row_bytes + tile - 1) / tile;
    per_group[jobs[i].k > jobs[i].p][jobs[i].p] += n;
    nitems += n;
  }
  if (nitems > kNoAllocItems)
    return fail(RAID6C_E_ARG, "%zu column tiles: at most %zu without allocation", nitems, kNoAllocItems);
  if (njobs == 0) return RAID6C_OK;

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(RAID6C_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(RAID6C_E_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);

  std::lock_guard<std::mutex> lk(g_mu);
  uint8_t* d_scratch = nullptr;
  const int rc = scratch_on(dev, &d_scratch);
  if (rc != RAID6C_OK) return rc;

  // Items grouped by prime, largest prime first, plain before extended (as a
  // plan's grouped schedule orders them); first[x][p] is where group (p, x)
  // starts.
  size_t first[2][kMaxPrime + 1] = {};
  size_t pos = 0;
  for (int p = kMaxPrime; p >= 3; --p)
    for (int x = 0; x < 2; ++x) {
      first[x][p] = pos;
      pos += per_group[x][p];
    }
  size_t fill[2][kMaxPrime + 1];
  memcpy(fill, first, sizeof fill);
  for (size_t i = 0; i < njobs; ++i) {
    Case cs;
    (void)check_job(jobs[i], i, &cs);
    g_jobs[i] = make_batch_job(jobs[i], cs);
    const int p = jobs[i].p, x = jobs[i].k > p;
    const uint32_t tile = 64u * 4u * (uint32_t)zp_prime_entry(p)->group_vec;
    for (uint32_t c = 0; c < jobs[i].row_bytes; c += tile) g_items[fill[x][p]++] = BatchItem{(uint32_t)i, c};
  }

  const hipStream_t s = (hipStream_t)stream;
  const BatchJob* d_jobs = (const BatchJob*)d_scratch;
  const BatchItem* d_items = (const BatchItem*)(d_scratch + kJobsBytes);
  if ((e = hipMemcpyAsync((void*)d_jobs, g_jobs, njobs * sizeof(BatchJob), hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync((void*)d_items, g_items, nitems * sizeof(BatchItem), hipMemcpyHostToDevice, s)) != hipSuccess)
    return fail(RAID6C_E_HIP, "table upload: %s", hipGetErrorString(e));
  for (int p = kMaxPrime; p >= 3; --p)
    for (int x = 0; x < 2; ++x) {
      const size_t n = per_group[x][p];
      if (n == 0) continue;
      const ZpPrimeEntry* pe = zp_prime_entry(p);
      GroupArgs ga{d_jobs, d_items + first[x][p], (uint32_t)n};
      void* args[] = {(void*)&ga};
      const unsigned grid = (unsigned)((n + pe->group_per_wg - 1) / pe->group_per_wg);
      e = hipLaunchKernel(x ? pe->group_ext_kernel : pe->group_kernel, dim3(grid), dim3(pe->group_threads), args,
                          (size_t)pe->group_lds, s);
      if (e != hipSuccess) return fail(RAID6C_E_HIP, "job-list launch (p = %d): %s", p, hipGetErrorString(e));
    }
  return RAID6C_OK;
}
