// batch.hip -- plans: stripes of mixed p, k and row size, encoded and
// recovered in one HIP graph launch, replayed any number of times.
//
// Two schedules:
//  * grouped (the default): the jobs of each prime form one grid of that
//    prime's job-list kernel (zp_kernels.hip, variant 3), one column tile
//    per wave, with the prime's own register budget and vector width.  The
//    grids are the graph's nodes, independent (grouped = 1) or chained one
//    after another (grouped = 2).
//  * persistent (grouped = 0): items of one wavefront each, 64 lanes x 4
//    bytes = a 256-byte column tile of one stripe.  A persistent grid of
//    single-wave work-groups pops items from a device counter (a chunk at a
//    time) and runs the same per-tile code as the plain kernels
//    (tile_recover: encode is the "P and Q erased" case), dispatched on the
//    stripe's prime.  Items are ordered largest-first so the tail of the
//    launch is made of small items.  The graph holds two nodes: a one-thread
//    kernel that zeroes the counter (a kernel, not a memset node) and the
//    persistent kernel.  (The request server launches the kernel directly
//    and instead advances the counter's base by the exact number of
//    increments each run takes.)
#include <hip/hip_runtime.h>

#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <vector>

#include "../../include/raid6c.h"
#include "raid6c_internal.h"
#include "zp_core.hpp"

namespace raid6c {

int fail(int code, const char* fmt, ...);

namespace {

constexpr int kLanes = 64;
constexpr int kTileBytes = kBatchTileBytes;
static_assert(kTileBytes == kLanes * 4, "one dword per lane and row");

// Strips whose loads are batched per prime: as many as fit beside the
// (2p-1) accumulator dwords in the register budget set by the largest prime
// (about 160 dwords), never more than p.
constexpr int batch_unroll(int p) {
  const int cap = (160 - (2 * p - 1)) / (p - 1);
  const int u = cap < 1 ? 1 : cap;
  return u > p ? p : u;
}

// Jobs whose rows are not all on 128-byte lines load with the ordinary
// cache policy, as in the job-list kernels: the line at the edge of two
// tiles is then still cached for the second reader (all non-temporal, the
// 20,000-stripe mix took 31.0 ms; with the choice per job, 27.6 ms).
template <int P>
__device__ __forceinline__ void run_item(const BatchJob& j, uint32_t col, uint32_t* lds) {
  const ColsJob c{j.base, j.strip_stride, j.out0, j.out1, j.src, j.src_stride, j.e0, j.e1,
                  j.row_bytes, col, (uint32_t)((P - 1) * j.row_bytes)};
  const Case cs{j.op, j.x, j.y};
  if (c.lines_aligned())
    tile_recover<P, 1, batch_unroll(P), false>(c, j.k, cs, lds, kLanes);
  else
    tile_recover<P, 1, batch_unroll(P), false>(c.with_policy<kLoadPolicyShared>(), j.k, cs, lds, kLanes);
}

__global__ void reset_counter(uint64_t* counter) { *counter = 0ull; }

__global__ void __launch_bounds__(64) batch_kernel(const BatchArgs a) {
  extern __shared__ __align__(16) uint32_t smem[];
  const uint32_t lane = threadIdx.x;
  uint32_t* lds = smem + lane;
  for (;;) {
    uint32_t got = 0;
    if (lane == 0) {
      const uint64_t v = atomicAdd((unsigned long long*)a.counter, (unsigned long long)a.chunk) - a.base;
      got = v < a.nitems ? (uint32_t)v : a.nitems;
    }
    const uint32_t first = __builtin_amdgcn_readfirstlane(got);
    if (first >= a.nitems) break;
    const uint32_t last = min(first + a.chunk, a.nitems);
    for (uint32_t it = first; it < last; ++it) {
      const BatchItem item = a.items[it];
      const BatchJob j = a.jobs[item.job];
      const uint32_t col = item.col + lane * 4u;
      if (col >= j.row_bytes) continue;
      switch (j.p) {
#define RAID6C_BATCH_CASE(q) \
  case q:                    \
    run_item<q>(j, col, lds); \
    break;
        RAID6C_BATCH_CASE(3)
        RAID6C_BATCH_CASE(5)
        RAID6C_BATCH_CASE(7)
        RAID6C_BATCH_CASE(11)
        RAID6C_BATCH_CASE(13)
        RAID6C_BATCH_CASE(17)
        RAID6C_BATCH_CASE(19)
        RAID6C_BATCH_CASE(23)
        RAID6C_BATCH_CASE(29)
        RAID6C_BATCH_CASE(31)
        RAID6C_BATCH_CASE(37)
        RAID6C_BATCH_CASE(41)
        RAID6C_BATCH_CASE(43)
        RAID6C_BATCH_CASE(47)
        RAID6C_BATCH_CASE(53)
        RAID6C_BATCH_CASE(59)
        RAID6C_BATCH_CASE(61)
#undef RAID6C_BATCH_CASE
        default:
          break;
      }
    }
  }
}

}  // namespace

hipError_t batch_launch(const BatchArgs& a, int grid, int max_p, hipStream_t stream) {
  hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(kLanes), (size_t)max_p * kLanes * 4, stream, a);
  return hipGetLastError();
}

const void* batch_kernel_fn() { return (const void*)batch_kernel; }
const void* batch_reset_fn() { return (const void*)reset_counter; }

namespace {

bool is_odd_prime(int p) {
  if (p < 3 || (p % 2) == 0) return false;
  for (int d = 3; d * d <= p; d += 2)
    if (p % d == 0) return false;
  return true;
}

}  // namespace

}  // namespace raid6c

using namespace raid6c;

struct raid6c_plan {
  int device = 0;
  std::vector<BatchJob> jobs;
  std::vector<BatchItem> items;   // current order (persistent kernel, 256-byte tiles)
  std::vector<uint64_t> job_cost; // bytes moved per tile, per job
  void* dmem = nullptr;           // jobs | items | counter | group items
  BatchArgs args{};
  // Grouped schedule: one job-list grid per prime, as independent graph nodes.
  struct Group {
    int p;
    bool ext;                     // jobs with the extended Q parity (k > p)
    uint32_t first, n;            // range in gitems
  };
  bool has_ext = false;           // some job has k > p: grouped schedules only
  std::vector<BatchItem> gitems;  // per prime, tiles of 64 lanes x that prime's group_vec dwords
  std::vector<Group> groups;
  std::vector<GroupArgs> gargs;
  const BatchItem* d_gitems = nullptr;
  int max_p = 3;
  int cus = 256;
  raid6c_schedule sched{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t bytes = 0;             // algorithmic bytes per run
  uint64_t user_bytes = 0;
};

namespace {

void order_items(raid6c_plan* pl, int order) {
  const size_t nj = pl->jobs.size();
  std::vector<uint32_t> idx(nj);
  for (size_t i = 0; i < nj; ++i) idx[i] = (uint32_t)i;
  if (order == RAID6C_ORDER_LARGEST_FIRST) {
    std::stable_sort(idx.begin(), idx.end(),
                     [&](uint32_t a, uint32_t b) { return pl->job_cost[a] > pl->job_cost[b]; });
  } else if (order == RAID6C_ORDER_BY_PRIME) {
    std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) {
      if (pl->jobs[a].p != pl->jobs[b].p) return pl->jobs[a].p > pl->jobs[b].p;
      return pl->job_cost[a] > pl->job_cost[b];
    });
  }
  pl->items.clear();
  for (uint32_t j : idx) {
    const uint32_t w = pl->jobs[j].row_bytes;
    for (uint32_t c = 0; c < w; c += kTileBytes) pl->items.push_back(BatchItem{j, c});
  }
}

// Items of the grouped schedule: jobs of one prime, and of one code (plain,
// or extended Q parity), together (largest p first, plain before extended,
// costliest stripes first within a group), each job's tiles consecutive.
void group_items(raid6c_plan* pl) {
  const size_t nj = pl->jobs.size();
  std::vector<uint32_t> idx(nj);
  for (size_t i = 0; i < nj; ++i) idx[i] = (uint32_t)i;
  auto ext = [&](uint32_t j) { return pl->jobs[j].k > pl->jobs[j].p; };
  std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) {
    if (pl->jobs[a].p != pl->jobs[b].p) return pl->jobs[a].p > pl->jobs[b].p;
    if (ext(a) != ext(b)) return !ext(a);
    return pl->job_cost[a] > pl->job_cost[b];
  });
  pl->gitems.clear();
  pl->groups.clear();
  for (uint32_t j : idx) {
    const int p = pl->jobs[j].p;
    if (pl->groups.empty() || pl->groups.back().p != p || pl->groups.back().ext != ext(j))
      pl->groups.push_back(raid6c_plan::Group{p, ext(j), (uint32_t)pl->gitems.size(), 0});
    const uint32_t tile = 64u * 4u * (uint32_t)zp_prime_entry(p)->group_vec;
    const uint32_t w = pl->jobs[j].row_bytes;
    for (uint32_t c = 0; c < w; c += tile) pl->gitems.push_back(BatchItem{j, c});
    pl->groups.back().n = (uint32_t)pl->gitems.size() - pl->groups.back().first;
  }
}

void free_graph(raid6c_plan* pl) {
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  pl->exec = nullptr;
  pl->graph = nullptr;
}

// Upload the item order and (re)build the two-node graph for the current
// schedule.
int build_graph(raid6c_plan* pl) {
  free_graph(pl);
  hipError_t e;
  if ((e = hipGraphCreate(&pl->graph, 0)) != hipSuccess)
    return fail(RAID6C_E_HIP, "hipGraphCreate: %s", hipGetErrorString(e));
  if (pl->sched.grouped) {
    // One node per prime: no edges (grouped = 1), so the grids may run side
    // by side, or a chain (grouped = 2), largest prime first.
    pl->gargs.clear();
    for (const auto& g : pl->groups) pl->gargs.push_back(GroupArgs{pl->args.jobs, pl->d_gitems + g.first, g.n});
    hipGraphNode_t prev = nullptr;
    for (size_t gi = 0; gi < pl->groups.size(); ++gi) {
      const raid6c_plan::Group& g = pl->groups[gi];
      hipGraphNode_t node;
      const bool chain = pl->sched.grouped == 2 && prev != nullptr;
      void* params[] = {(void*)&pl->gargs[gi]};
      hipKernelNodeParams kp{};
      const ZpPrimeEntry* pe = zp_prime_entry(g.p);
      kp.func = (void*)(g.ext ? pe->group_ext_kernel : pe->group_kernel);
      kp.gridDim = dim3((g.n + pe->group_per_wg - 1) / pe->group_per_wg);
      kp.blockDim = dim3(pe->group_threads);
      kp.sharedMemBytes = (unsigned)pe->group_lds;
      kp.kernelParams = params;
      if ((e = hipGraphAddKernelNode(&node, pl->graph, chain ? &prev : nullptr, chain ? 1 : 0, &kp)) != hipSuccess)
        return fail(RAID6C_E_HIP, "hipGraphAddKernelNode: %s", hipGetErrorString(e));
      prev = node;
    }
    if ((e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0)) != hipSuccess)
      return fail(RAID6C_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    return RAID6C_OK;
  }
  e = hipMemcpy((void*)pl->args.items, pl->items.data(), pl->items.size() * sizeof(BatchItem),
                hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(RAID6C_E_HIP, "plan upload failed: %s", hipGetErrorString(e));
  pl->args.chunk = (uint32_t)pl->sched.chunk;

  hipGraphNode_t reset_node, batch_node;
  void* reset_params[] = {(void*)&pl->args.counter};
  hipKernelNodeParams rp{};
  rp.func = (void*)batch_reset_fn();
  rp.gridDim = dim3(1);
  rp.blockDim = dim3(1);
  rp.sharedMemBytes = 0;
  rp.kernelParams = reset_params;
  if ((e = hipGraphAddKernelNode(&reset_node, pl->graph, nullptr, 0, &rp)) != hipSuccess)
    return fail(RAID6C_E_HIP, "hipGraphAddKernelNode: %s", hipGetErrorString(e));

  void* batch_params[] = {(void*)&pl->args};
  hipKernelNodeParams bp{};
  bp.func = (void*)batch_kernel_fn();
  bp.gridDim = dim3((unsigned)(pl->cus * pl->sched.waves_per_cu));
  bp.blockDim = dim3(kLanes);
  bp.sharedMemBytes = (unsigned)(pl->max_p * kLanes * 4);
  bp.kernelParams = batch_params;
  if ((e = hipGraphAddKernelNode(&batch_node, pl->graph, &reset_node, 1, &bp)) != hipSuccess)
    return fail(RAID6C_E_HIP, "hipGraphAddKernelNode: %s", hipGetErrorString(e));
  if ((e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0)) != hipSuccess)
    return fail(RAID6C_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  return RAID6C_OK;
}

}  // namespace

int raid6c::check_job(const raid6c_job& J, size_t i, Case* out) {
  const int p = J.p, k = J.k;
  if (!is_odd_prime(p)) return fail(RAID6C_E_ARG, "job %zu: p = %d is not an odd prime", i, p);
  if (p > kMaxPrime) return fail(RAID6C_E_UNSUPPORTED, "job %zu: p = %d is not built", i, p);
  const int kmax = raid6c_max_data_strips(p);
  if (k < 1 || k > kmax)
    return fail(RAID6C_E_ARG, "job %zu: k = %d not in [1, %d]%s", i, k, kmax,
                kmax == p ? " (p fails Theorem 3.3.3: no extended Q parity)" : "");
  if (J.row_bytes == 0 || (J.row_bytes % 16) != 0)
    return fail(RAID6C_E_ARG, "job %zu: row_bytes must be a positive multiple of 16", i);
  if ((uint64_t)(p - 1) * J.row_bytes >= (1ull << 31)) return fail(RAID6C_E_ARG, "job %zu: strip of 2 GiB or more", i);
  if (J.base == nullptr || ((uintptr_t)J.base & 15u) != 0)
    return fail(RAID6C_E_ARG, "job %zu: base is NULL or not 16-byte aligned", i);
  if ((J.strip_stride % 16) != 0 || J.strip_stride < (uint64_t)(p - 1) * J.row_bytes)
    return fail(RAID6C_E_ARG, "job %zu: bad strip_stride", i);
  if (J.op != RAID6C_JOB_ENCODE && J.op != RAID6C_JOB_RECOVER)
    return fail(RAID6C_E_ARG, "job %zu: op must be encode or recover", i);
  Case cs{OP_PQ, -1, -1};
  if (J.op == RAID6C_JOB_RECOVER) {
    cs = classify(k, J.e0, J.e1);
    if (cs.op == OP_BAD) return fail(RAID6C_E_ARG, "job %zu: invalid erasures (%d, %d)", i, J.e0, J.e1);
  }
  *out = cs;
  return RAID6C_OK;
}

BatchJob raid6c::make_batch_job(const raid6c_job& J, const Case& cs) {
  BatchJob b{};
  b.base = (uint8_t*)J.base;
  b.strip_stride = J.strip_stride;
  b.row_bytes = J.row_bytes;
  b.p = (int16_t)J.p;
  b.k = (int16_t)J.k;
  b.op = (int16_t)cs.op;
  b.x = (int16_t)cs.x;
  b.y = (int16_t)cs.y;
  b.e0 = -1;
  b.e1 = -1;
  b.src = nullptr;
  return b;
}

namespace {

bool valid_schedule(const raid6c_schedule& s) {
  return s.waves_per_cu >= 1 && s.waves_per_cu <= 32 && s.chunk >= 1 && s.chunk <= 1024 &&
         (s.order == RAID6C_ORDER_LARGEST_FIRST || s.order == RAID6C_ORDER_BY_PRIME ||
          s.order == RAID6C_ORDER_SUBMITTED) &&
         (s.grouped == 0 || s.grouped == 1 || s.grouped == 2);
}

}  // namespace

extern "C" {

int raid6c_plan_create(const raid6c_job* jobs, size_t njobs, raid6c_plan** out) {
  if (out == nullptr) return fail(RAID6C_E_ARG, "out is NULL");
  *out = nullptr;
  if (jobs == nullptr && njobs != 0) return fail(RAID6C_E_ARG, "jobs is NULL");
  if (njobs > 0xFFFFFFFFull) return fail(RAID6C_E_ARG, "too many jobs");
  raid6c_plan* pl = new (std::nothrow) raid6c_plan();
  if (pl == nullptr) return fail(RAID6C_E_NOMEM, "out of host memory");

  // Check every job and every strip interval (no two jobs may share bytes).
  struct Span {
    uintptr_t lo, hi;
    uint32_t job;
  };
  std::vector<Span> spans;
  pl->jobs.reserve(njobs);
  for (size_t i = 0; i < njobs; ++i) {
    const raid6c_job& J = jobs[i];
    const int p = J.p, k = J.k;
    Case cs{OP_PQ, -1, -1};
    const int rc = check_job(J, i, &cs);
    if (rc != RAID6C_OK) {
      delete pl;
      return rc;
    }
    pl->jobs.push_back(make_batch_job(J, cs));
    if (k > p) pl->has_ext = true;
    const uint64_t strip = (uint64_t)(p - 1) * J.row_bytes;
    const int moved = (cs.op == OP_P || cs.op == OP_Q || cs.op == OP_D) ? k + 1 : k + 2;
    pl->bytes += (uint64_t)moved * strip;
    pl->user_bytes += (uint64_t)k * strip;
    pl->job_cost.push_back((uint64_t)moved * (p - 1));
    if (p > pl->max_p) pl->max_p = p;
    for (int j = 0; j < k + 2; ++j) {
      const uintptr_t lo = (uintptr_t)J.base + (uintptr_t)j * J.strip_stride;
      spans.push_back(Span{lo, lo + (uintptr_t)strip, (uint32_t)i});
    }
  }
  std::sort(spans.begin(), spans.end(), [](const Span& a, const Span& b) { return a.lo < b.lo; });
  uintptr_t reach = 0;
  uint32_t reach_job = 0;
  for (size_t i = 0; i < spans.size(); ++i) {
    if (i > 0 && spans[i].lo < reach) {
      const int rc = fail(RAID6C_E_ARG, "strips of jobs %u and %u overlap", reach_job, spans[i].job);
      delete pl;
      return rc;
    }
    if (spans[i].hi > reach) {
      reach = spans[i].hi;
      reach_job = spans[i].job;
    }
  }

  (void)hipGetDevice(&pl->device);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl->device) == hipSuccess && cus > 0)
    pl->cus = cus;
  // Default: the per-prime grids one after another (on the 20,000-stripe
  // mix 21.4 ms against 22.4 ms side by side).
  pl->sched = raid6c_schedule{8, 4, RAID6C_ORDER_LARGEST_FIRST, 2};
  order_items(pl, pl->sched.order);
  group_items(pl);
  if (pl->items.size() > 0xFFFFFFFFull || pl->gitems.size() > 0xFFFFFFFFull) {
    delete pl;
    return fail(RAID6C_E_ARG, "too many work items");
  }

  const size_t jb = std::max<size_t>(1, pl->jobs.size()) * sizeof(BatchJob);
  const size_t ib = std::max<size_t>(1, pl->items.size()) * sizeof(BatchItem);
  const size_t gb = std::max<size_t>(1, pl->gitems.size()) * sizeof(BatchItem);
  const size_t total = jb + ib + 256 + gb;
  hipError_t e = hipMalloc(&pl->dmem, total);
  if (e != hipSuccess) {
    delete pl;
    return fail(RAID6C_E_NOMEM, "hipMalloc of %zu bytes failed: %s", total, hipGetErrorString(e));
  }
  pl->args.jobs = (const BatchJob*)pl->dmem;
  pl->args.items = (const BatchItem*)((uint8_t*)pl->dmem + jb);
  pl->args.counter = (uint64_t*)((uint8_t*)pl->dmem + jb + ib);
  pl->d_gitems = (const BatchItem*)((uint8_t*)pl->dmem + jb + ib + 256);
  pl->args.base = 0;
  pl->args.nitems = (uint32_t)pl->items.size();
  if ((!pl->jobs.empty() &&
       (e = hipMemcpy((void*)pl->args.jobs, pl->jobs.data(), pl->jobs.size() * sizeof(BatchJob),
                      hipMemcpyHostToDevice)) != hipSuccess) ||
      (!pl->gitems.empty() &&
       (e = hipMemcpy((void*)pl->d_gitems, pl->gitems.data(), pl->gitems.size() * sizeof(BatchItem),
                      hipMemcpyHostToDevice)) != hipSuccess)) {
    (void)hipFree(pl->dmem);
    delete pl;
    return fail(RAID6C_E_HIP, "plan upload failed: %s", hipGetErrorString(e));
  }
  const int rc = build_graph(pl);
  if (rc != RAID6C_OK) {
    raid6c_plan_destroy(pl);
    return rc;
  }
  *out = pl;
  return RAID6C_OK;
}

int raid6c_plan_run(raid6c_plan* plan, void* stream) {
  if (plan == nullptr) return fail(RAID6C_E_ARG, "plan is NULL");
  if (plan->items.empty()) return RAID6C_OK;
  const hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
  if (e != hipSuccess) return fail(RAID6C_E_HIP, "hipGraphLaunch: %s", hipGetErrorString(e));
  return RAID6C_OK;
}

int raid6c_plan_get_schedule(const raid6c_plan* plan, raid6c_schedule* out) {
  if (plan == nullptr || out == nullptr) return fail(RAID6C_E_ARG, "NULL argument");
  *out = plan->sched;
  return RAID6C_OK;
}

int raid6c_plan_set_schedule(raid6c_plan* plan, const raid6c_schedule* s) {
  if (plan == nullptr || s == nullptr) return fail(RAID6C_E_ARG, "NULL argument");
  if (!valid_schedule(*s)) return fail(RAID6C_E_ARG, "invalid schedule");
  if (s->grouped == 0 && plan->has_ext)
    return fail(RAID6C_E_UNSUPPORTED, "the persistent kernel runs the plain code only (a job has k > p)");
  const bool reorder = s->order != plan->sched.order;
  // A persistent-kernel replay reads the item order from device memory:
  // finish the runs in flight before it is rewritten.
  if (reorder) (void)hipDeviceSynchronize();
  plan->sched = *s;
  if (reorder) order_items(plan, s->order);
  return build_graph(plan);
}

int raid6c_plan_stats(const raid6c_plan* plan, raid6c_plan_info* out) {
  if (plan == nullptr || out == nullptr) return fail(RAID6C_E_ARG, "NULL argument");
  out->njobs = plan->jobs.size();
  out->nitems = plan->items.size();
  out->bytes_moved = plan->bytes;
  out->user_bytes = plan->user_bytes;
  out->max_p = plan->max_p;
  uint64_t wgs = 0;
  for (const auto& g : plan->groups) {
    const int per = zp_prime_entry(g.p)->group_per_wg;
    wgs += (g.n + per - 1) / per;
  }
  out->grid = plan->sched.grouped ? (uint32_t)wgs : (uint32_t)(plan->cus * plan->sched.waves_per_cu);
  return RAID6C_OK;
}

int raid6c_plan_autotune(raid6c_plan* plan, void* stream, int reps, float* best_ms) {
  if (plan == nullptr) return fail(RAID6C_E_ARG, "plan is NULL");
  if (reps < 1 || reps > 1000) return fail(RAID6C_E_ARG, "reps must be in [1, 1000]");
  if (plan->items.empty()) {
    if (best_ms) *best_ms = 0.f;
    return RAID6C_OK;
  }
  const hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(RAID6C_E_HIP, "hipEventCreate failed");
  const int waves[] = {4, 8, 12, 16};
  const int chunks[] = {1, 4, 16};
  const int orders[] = {RAID6C_ORDER_LARGEST_FIRST, RAID6C_ORDER_BY_PRIME};
  raid6c_schedule best = plan->sched;
  float best_t = 1e30f;
  int rc = RAID6C_OK;
  // The two grouped schedules, then every persistent-kernel candidate (plain
  // code only).
  const int ncand = plan->has_ext ? 2 : 2 + 2 * 4 * 3;
  for (int gi = 0; gi < ncand; ++gi) {
    {
      {
        const raid6c_schedule cand = gi < 2 ? raid6c_schedule{8, 4, RAID6C_ORDER_LARGEST_FIRST, 1 + gi}
                                            : raid6c_schedule{waves[((gi - 2) / 3) % 4], chunks[(gi - 2) % 3],
                                                              orders[(gi - 2) / 12], 0};
        if ((rc = raid6c_plan_set_schedule(plan, &cand)) != RAID6C_OK) goto done;
        if ((rc = raid6c_plan_run(plan, stream)) != RAID6C_OK) goto done;  // warm-up
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r)
          if ((rc = raid6c_plan_run(plan, stream)) != RAID6C_OK) goto done;
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) {
          rc = fail(RAID6C_E_HIP, "hipEventSynchronize failed");
          goto done;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= (float)reps;
        if (ms < best_t) {
          best_t = ms;
          best = cand;
        }
      }
    }
  }
  rc = raid6c_plan_set_schedule(plan, &best);
  if (best_ms) *best_ms = best_t;
done:
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int raid6c_run_jobs(const raid6c_job* jobs, size_t njobs, void* stream) {
  if (jobs == nullptr && njobs != 0) return fail(RAID6C_E_ARG, "jobs is NULL");
  for (size_t i = 0; i < njobs; ++i) {
    Case cs;
    const int rc = check_job(jobs[i], i, &cs);
    if (rc != RAID6C_OK) return rc;
  }
  for (size_t i = 0; i < njobs; ++i) {
    const raid6c_job& J = jobs[i];
    int rc;
    if (J.op == RAID6C_JOB_ENCODE) {
      rc = raid6c_encode_n(J.p, J.k, J.row_bytes, J.base, J.strip_stride, (size_t)(J.k + 2) * J.strip_stride, 1,
                           stream);
    } else {
      void* strips[kMaxStrips];
      for (int j = 0; j < J.k + 2; ++j) strips[j] = (uint8_t*)J.base + (size_t)j * J.strip_stride;
      rc = (J.e1 < 0) ? raid6c_recover_1(J.p, J.k, J.row_bytes, strips, J.e0, stream)
                      : raid6c_recover_2(J.p, J.k, J.row_bytes, strips, J.e0, J.e1, stream);
    }
    if (rc != RAID6C_OK) return rc;
  }
  return RAID6C_OK;
}

int raid6c_plan_destroy(raid6c_plan* plan) {
  if (plan == nullptr) return RAID6C_OK;
  free_graph(plan);
  if (plan->dmem) (void)hipFree(plan->dmem);
  delete plan;
  return RAID6C_OK;
}

}  // extern "C"
