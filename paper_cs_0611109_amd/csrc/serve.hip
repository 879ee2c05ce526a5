// serve.hip -- a request server with continuous batching.
//
// Clients submit writes (a payload becomes a new resident stripe: data strips
// copied into the store and P, Q computed in the same pass) and degraded
// reads (one or two strips of a resident stripe rebuilt into a client
// buffer).  The stripe store is one device allocation (the HBM budget) used
// as a ring: stripes are placed in arrival order and the oldest idle stripes
// are evicted when a write needs room.
//
// A scheduler thread admits pending requests into free "slots" (a stream, an
// event and job/item tables) and launches each slot's requests as one grid
// of the job-list kernel per prime present (a plan's grouped schedule; small
// groups of the primes up to 31 share one grid of the multi-prime kernel,
// zp_multi.hip), or, with `persistent` set, as one persistent kernel
// (batch.hip); requests that arrive
// while slots are busy are admitted into the next free slot, so up to
// max_inflight batches overlap on the device.  A completion thread polls the
// slots' events, stamps completion times and releases stripes.  With
// `plain` set, every request is instead one plain launch (raid6c_write /
// raid6c_read_degraded) on a single stream: the per-request path.
//
// A degraded read of a stripe whose write is admitted in the same batch runs
// in the batch's second launch phase, after the first phase that holds the
// write; a read of a stripe whose write is in another slot's batch in flight
// is parked on the host until that write completes (waiting on the device
// would hold the read's whole batch behind the other one).
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_set>
#include <vector>

#include "../../include/raid6c.h"
#include "raid6c_internal.h"
#include "stripe_index.h"
#include "zp_multi.h"

namespace raid6c {
int fail(int code, const char* fmt, ...);
}

using namespace raid6c;

namespace {

using Clock = std::chrono::steady_clock;

bool is_odd_prime(int p) {
  if (p < 3 || (p % 2) == 0) return false;
  for (int d = 3; d * d <= p; d += 2)
    if (p % d == 0) return false;
  return true;
}

uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Groups of a batch with fewer 256-byte column tiles than this (a few per
// SIMD of the GPU) run the job-list kernel set for latency.
#ifndef RAID6C_LATENCY_TILES
#define RAID6C_LATENCY_TILES 4096
#endif
constexpr size_t kLatencyTiles = RAID6C_LATENCY_TILES;

// Largest batch formed while no other batch is in flight.
constexpr size_t kIdleBatch = 128;

// Small groups of primes up to kMultiMaxPrime share one grid per phase.
#ifndef RAID6C_SERVE_MULTI
#define RAID6C_SERVE_MULTI 1
#endif
constexpr bool kMultiGrids = RAID6C_SERVE_MULTI != 0;

struct Pending {
  raid6c_request req;
  uint64_t arrival_ns;
  size_t index;    // position in a replay, else SIZE_MAX
};

struct Slot;

struct Resident {
  uint64_t id;
  uint64_t off;    // byte offset in the store
  uint64_t bytes;  // reserved bytes
  int p, k;
  uint32_t row_bytes;
  int refs;        // admitted requests not yet complete
  bool ready;      // its write has completed
  bool failed;     // its write could not be launched: reads of it are invalid
  Slot* writer;    // the slot whose batch writes it, while that is in flight
  std::vector<Pending> waiters;  // reads parked until that write completes
};

struct InFlight {
  raid6c_request req;
  uint64_t arrival_ns;
  size_t index;
  Resident* stripe;
  int phase;       // 1: a read of a stripe written in the same batch (runs after phase 0)
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  uint8_t* h_buf = nullptr;     // pinned: items | jobs of the batch being formed
  uint8_t* d_mem = nullptr;     // counter (256 bytes) | items | jobs
  size_t cap = 0;               // bytes of h_buf and of d_mem's table area
  uint64_t counter = 0;         // value the device counter holds between runs
  std::vector<InFlight> reqs;
  size_t items = 0;       // 256-byte column tiles of reqs (for the tables)
  uint64_t launch_ns = 0;
  bool busy = false;      // owns requests
  bool launched = false;  // its completion event has been recorded
  std::vector<uint8_t*> retired_h, retired_d;  // outgrown tables, freed at destroy
};

}  // namespace

struct raid6c_server {
  raid6c_server_config cfg{};
  int device = 0;
  int cus = 256;
  uint8_t* store = nullptr;
  uint64_t head = 0;             // next free byte (ring)
  std::deque<Resident*> fifo;    // resident stripes, oldest first
  StripeIndex<Resident> index{8192};  // the same stripes by id
  std::deque<Resident> pool;     // records (stable addresses), reused through free_res
  std::vector<Resident*> free_res;
  std::vector<Slot> slots;
  hipStream_t plain_stream = nullptr;

  std::mutex mu;
  std::condition_variable cv_sched;  // pending work or a free slot
  std::condition_variable cv_done;   // completions
  std::deque<Pending> pending;
  std::deque<raid6c_completion> done;
  size_t parked = 0;                 // reads waiting in a stripe's waiters
  raid6c_completion* replay_out = nullptr;
  size_t outstanding = 0;            // submitted, not complete
  bool stopping = false;
  raid6c_server_stats stats{};
  Clock::time_point t0 = Clock::now();
  std::thread scheduler, completer;
  int thread_error = 0;

  uint64_t now_ns() const {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count();
  }
};

namespace {

uint64_t stripe_bytes(int p, int k, uint32_t w) { return round_up((uint64_t)(k + 2) * (p - 1) * w, 256); }

int check_request(const raid6c_request& r) {
  if (r.kind != RAID6C_REQ_WRITE && r.kind != RAID6C_REQ_READ) return RAID6C_ST_INVALID;
  if (r.kind == RAID6C_REQ_READ) return RAID6C_ST_OK;  // geometry comes from the stripe
  if (!is_odd_prime(r.p) || r.p > kMaxPrime || r.k < 1 || r.k > raid6c_max_data_strips(r.p))
    return RAID6C_ST_INVALID;
  if (r.row_bytes == 0 || (r.row_bytes % 16) != 0) return RAID6C_ST_INVALID;
  if ((uint64_t)(r.p - 1) * r.row_bytes >= (1ull << 31)) return RAID6C_ST_INVALID;
  if (r.src == nullptr || ((uintptr_t)r.src & 15u) != 0) return RAID6C_ST_INVALID;
  return RAID6C_ST_OK;
}

// Place a new stripe in the ring (ring_fit), evicting the oldest idle
// stripes as needed.  Returns the stripe, or nullptr when it must wait (the
// oldest stripe is busy) or can never fit (*never = true).
Resident* place(raid6c_server* s, const raid6c_request& r, bool* never) {
  const uint64_t need = stripe_bytes(r.p, r.k, r.row_bytes);
  *never = need > s->cfg.store_bytes;
  if (*never) return nullptr;
  for (;;) {
    uint64_t off = 0;
    const bool fits = ring_fit(s->head, s->fifo.empty() ? 0 : s->fifo.front()->off, s->fifo.empty(), need,
                               s->cfg.store_bytes, &off);
    if (fits) {
      Resident* st;
      if (!s->free_res.empty()) {
        st = s->free_res.back();
        s->free_res.pop_back();
      } else {
        s->pool.emplace_back();
        st = &s->pool.back();
      }
      st->id = r.stripe_id;
      st->off = off;
      st->bytes = need;
      st->p = r.p;
      st->k = r.k;
      st->row_bytes = r.row_bytes;
      st->refs = 0;
      st->ready = st->failed = false;
      st->writer = nullptr;
      st->waiters.clear();
      s->fifo.push_back(st);
      s->index.insert(r.stripe_id, st);
      s->head = off + need;
      return st;
    }
    // Evict the oldest stripe if it is idle, else wait.
    Resident* oldest = s->fifo.front();
    if (oldest->refs > 0) return nullptr;
    s->fifo.pop_front();
    s->index.erase(oldest->id);
    s->free_res.push_back(oldest);
    s->stats.evictions++;
  }
}

void complete_one(raid6c_server* s, const raid6c_request& req, uint64_t arrival, size_t index, int status,
                  uint64_t launch_ns, uint64_t done_ns, int batch, uint64_t user_bytes = 0) {
  raid6c_completion c{};
  c.tag = req.tag;
  c.status = status;
  c.batch_size = batch;
  c.arrival_ns = arrival;
  c.launch_ns = launch_ns;
  c.complete_ns = done_ns;
  if (s->replay_out != nullptr && index != SIZE_MAX) s->replay_out[index] = c;
  else s->done.push_back(c);
  s->stats.completed++;
  if (status == RAID6C_ST_OK) s->stats.user_bytes += user_bytes;
  s->outstanding--;
}

size_t table_bytes(size_t jobs, size_t items) {
  return round_up(items * sizeof(BatchItem), 64) + jobs * sizeof(BatchJob);
}

// Make room for a batch's tables; a new device block starts with a zeroed
// counter.  Called without the lock, on the slot's stream being idle.  The
// first call sizes the tables exactly; later ones at least double them.  The
// outgrown buffers are kept until the server is destroyed: freeing them now
// would synchronise the whole device and stall every batch in flight.
bool grow_slot(Slot& sl, size_t jobs, size_t items, bool* grew = nullptr) {
  const size_t need = table_bytes(jobs, items);
  if (need <= sl.cap) return true;
  if (grew != nullptr) *grew = sl.cap != 0;
  const size_t cap = sl.cap == 0 ? need : std::max(need, sl.cap * 2);
  if (sl.h_buf) sl.retired_h.push_back(sl.h_buf);
  if (sl.d_mem) sl.retired_d.push_back(sl.d_mem);
  sl.h_buf = nullptr;
  sl.d_mem = nullptr;
  sl.cap = 0;
  if (hipHostMalloc((void**)&sl.h_buf, cap, 0) != hipSuccess) return false;
  if (hipMalloc((void**)&sl.d_mem, cap + 256) != hipSuccess) return false;
  if (hipMemsetAsync(sl.d_mem, 0, 256, sl.stream) != hipSuccess) return false;
  sl.counter = 0;
  sl.cap = cap;
  return true;
}

// The plan job of one admitted request.
void fill_job(const raid6c_server* s, const InFlight& f, BatchJob& j) {
  const Resident* st = f.stripe;
  const size_t strip = (size_t)(st->p - 1) * st->row_bytes;
  memset(&j, 0, sizeof j);
  j.base = s->store + st->off;
  j.strip_stride = strip;
  j.row_bytes = st->row_bytes;
  j.p = (int16_t)st->p;
  j.k = (int16_t)st->k;
  j.e0 = j.e1 = -1;
  if (f.req.kind == RAID6C_REQ_WRITE) {
    j.op = OP_PQ;
    j.x = j.y = -1;
    j.src = (const uint8_t*)f.req.src;
    j.src_stride = strip;
  } else {
    const Case cs = classify(st->k, f.req.e0, f.req.e1);
    j.op = (int16_t)cs.op;
    j.x = (int16_t)cs.x;
    j.y = (int16_t)cs.y;
    const int lo = (f.req.e1 < 0 || f.req.e0 < f.req.e1) ? f.req.e0 : f.req.e1;
    const int hi = f.req.e1 < 0 ? -1 : (f.req.e0 < f.req.e1 ? f.req.e1 : f.req.e0);
    j.e0 = (int16_t)lo;
    j.out0 = (uint8_t*)f.req.dst;
    j.e1 = (int16_t)hi;
    j.out1 = (uint8_t*)f.req.dst + strip;
  }
}

// The reads parked on a stripe go back to the head of the queue, oldest
// first (its write has completed or failed).  Called with the lock held.
void release_waiters(raid6c_server* s, Resident* st) {
  std::vector<Pending>& w = st->waiters;
  for (auto pw = w.rbegin(); pw != w.rend(); ++pw) s->pending.push_front(*pw);
  s->parked -= w.size();
  w.clear();
}

// Launch one slot's requests.  Called without the lock.
hipError_t launch_slot(raid6c_server* s, Slot& sl) {
  if (s->cfg.plain) {
    // One plain launch per request, on one stream.
    for (const InFlight& f : sl.reqs) {
      const Resident* st = f.stripe;
      const size_t strip = (size_t)(st->p - 1) * st->row_bytes;
      void* strips[kMaxStrips];
      for (int j = 0; j < st->k + 2; ++j) strips[j] = s->store + st->off + (size_t)j * strip;
      int rc;
      if (f.req.kind == RAID6C_REQ_WRITE)
        rc = raid6c_write(st->p, st->k, st->row_bytes, f.req.src, strip, strips, sl.stream);
      else
        rc = raid6c_read_degraded(st->p, st->k, st->row_bytes, (const void* const*)strips, f.req.e0, f.req.e1,
                                  f.req.dst, sl.stream);
      if (rc != RAID6C_OK) return hipErrorLaunchFailure;
    }
    return hipEventRecord(sl.done, sl.stream);
  }
  // h_buf: the items (column tiles), then the jobs in request order.
  size_t nitems = 0;
  for (const InFlight& f : sl.reqs) nitems += (f.stripe->row_bytes + kBatchTileBytes - 1) / kBatchTileBytes;
  const size_t jobs_off = round_up(nitems * sizeof(BatchItem), 64);
  BatchItem* h_items = (BatchItem*)sl.h_buf;
  BatchJob* h_jobs = (BatchJob*)(sl.h_buf + jobs_off);
  for (size_t i = 0; i < sl.reqs.size(); ++i) fill_job(s, sl.reqs[i], h_jobs[i]);
  uint64_t* d_counter = (uint64_t*)sl.d_mem;
  uint8_t* d_tab = sl.d_mem + 256;
  const BatchJob* d_jobs = (const BatchJob*)(d_tab + jobs_off);
  const BatchItem* d_items = (const BatchItem*)d_tab;
  hipError_t e;
  // Per launch phase (0: everything but phase-1 reads; 1: reads of stripes
  // written in phase 0), grids of the job-list kernels (as in a plan's
  // grouped schedule): the requests of one prime and one code (plain, or
  // extended Q parity: k > p) form a grid, largest prime first; items are
  // that prime's tiles (at least kBatchTileBytes, so the table holds them).
  // With `persistent` set, the plain-code requests of a phase run as one
  // persistent kernel over 256-byte tiles instead (the persistent kernel runs
  // the plain code only); the extended-parity ones still go by grid.  A
  // plain-code group too small to fill the GPU takes the job-list kernel set
  // for latency (several waves per tile, each walking a share of the strips),
  // a larger one the plans' kernel (set for bandwidth).
  auto is_ext = [&](uint32_t i) { return sl.reqs[i].stripe->k > sl.reqs[i].stripe->p; };
  struct Group {
    const ZpPrimeEntry* pe;
    bool ext;
    size_t begin, end;        // its requests: order[begin, end)
    const void* fn;
    uint32_t tile;            // bytes of a column tile
    int per_wg, threads, lds; // launch shape
    uint32_t first, n;        // its items
  };
  struct Phase {
    std::vector<uint32_t> order;  // requests that go by grid
    std::vector<Group> groups;
    uint32_t pfirst = 0, pn = 0;  // persistent kernel's items
  };
  Phase ph[2];
  nitems = 0;
  for (int f = 0; f < 2; ++f) {
    Phase& P = ph[f];
    // Requests by key (largest prime first, plain code before extended),
    // in request order within a key: one counting pass, no comparisons.
    constexpr int kKeys = 2 * (kMaxPrime + 1);
    uint32_t start[kKeys + 1] = {};
    auto key = [&](uint32_t i) { return 2 * (kMaxPrime - sl.reqs[i].stripe->p) + (is_ext(i) ? 1 : 0); };
    auto by_grid = [&](uint32_t i) { return sl.reqs[i].phase == f && (!s->cfg.persistent || is_ext(i)); };
    for (uint32_t i = 0; i < (uint32_t)sl.reqs.size(); ++i)
      if (by_grid(i)) start[key(i) + 1]++;
    for (int c = 0; c < kKeys; ++c) start[c + 1] += start[c];
    P.order.resize(start[kKeys]);
    for (uint32_t i = 0; i < (uint32_t)sl.reqs.size(); ++i)
      if (by_grid(i)) P.order[start[key(i)]++] = i;
    for (size_t o = 0; o < P.order.size(); ++o) {
      const Resident* st = sl.reqs[P.order[o]].stripe;
      if (P.groups.empty() || P.groups.back().pe->p != st->p || P.groups.back().ext != is_ext(P.order[o]))
        P.groups.push_back(Group{zp_prime_entry(st->p), is_ext(P.order[o]), o, o, nullptr, 0, 0, 0, 0, 0, 0});
      P.groups.back().end = o + 1;
    }
    for (Group& g : P.groups) {
      size_t tiles256 = 0;
      for (size_t o = g.begin; o < g.end; ++o)
        tiles256 += (sl.reqs[P.order[o]].stripe->row_bytes + kBatchTileBytes - 1) / kBatchTileBytes;
      const bool lat = !g.ext && tiles256 < kLatencyTiles;
      g.fn = g.ext ? g.pe->group_ext_kernel : (lat ? g.pe->group_lat_kernel : g.pe->group_kernel);
      g.tile = 64u * 4u * (uint32_t)(g.ext ? g.pe->group_ext_vec : (lat ? g.pe->group_lat_vec : g.pe->group_vec));
      g.per_wg = lat ? 1 : g.pe->group_per_wg;
      g.threads = lat ? g.pe->group_lat_threads : g.pe->group_threads;
      g.lds = lat ? g.pe->group_lat_lds : g.pe->group_lds;
    }
    if (s->cfg.persistent) {
      // 256-byte tiles of the phase's plain-code requests, in request order.
      P.pfirst = (uint32_t)nitems;
      for (uint32_t i = 0; i < (uint32_t)sl.reqs.size(); ++i)
        if (sl.reqs[i].phase == f && !is_ext(i))
          for (uint32_t c = 0; c < sl.reqs[i].stripe->row_bytes; c += kBatchTileBytes)
            h_items[nitems++] = BatchItem{i, c};
      P.pn = (uint32_t)nitems - P.pfirst;
    }
    for (Group& g : P.groups) {
      g.first = (uint32_t)nitems;
      for (size_t o = g.begin; o < g.end; ++o)
        for (uint32_t c = 0; c < sl.reqs[P.order[o]].stripe->row_bytes; c += g.tile)
          h_items[nitems++] = BatchItem{P.order[o], c};
      g.n = (uint32_t)nitems - g.first;
    }
  }
  // One upload for both tables.
  e = hipMemcpyAsync(d_tab, sl.h_buf, jobs_off + sl.reqs.size() * sizeof(BatchJob), hipMemcpyHostToDevice,
                     sl.stream);
  if (e != hipSuccess) return e;
  int max_p = 3;
  for (const InFlight& f : sl.reqs) max_p = std::max(max_p, f.stripe->p);
  for (int f = 0; f < 2; ++f) {
    const Phase& P = ph[f];
    // Consecutive groups of primes up to kMultiMaxPrime that take the
    // latency kernel run as one grid of the multi-prime kernel: grids on a
    // stream run one after another, and these are each too small to fill
    // the GPU.  Their items are contiguous and their tiles the same width.
    auto multi_ok = [&](const Group& g) {
      return g.fn == g.pe->group_lat_kernel && g.pe->p <= kMultiMaxPrime &&
             g.tile == 256u * (uint32_t)zp_multi_vec(g.pe->p);
    };
    for (size_t gi = 0; gi < P.groups.size();) {
      const Group& g = P.groups[gi];
      size_t end = gi + 1;
      if (kMultiGrids && multi_ok(g))
        while (end < P.groups.size() && multi_ok(P.groups[end])) ++end;
      if (end - gi > 1) {
        const uint32_t n = P.groups[end - 1].first + P.groups[end - 1].n - g.first;
        int lds = 0;   // the largest need of the primes present (vec 2 stops at p = 13)
        for (size_t m = gi; m < end; ++m) lds = std::max(lds, zp_multi_lds(P.groups[m].pe->p));
        GroupArgs ga{d_jobs, d_items + g.first, n};
        void* args[] = {(void*)&ga};
        e = hipLaunchKernel(zp_multi_kernel(), dim3(n), dim3(256), args, (size_t)lds, sl.stream);
      } else {
        GroupArgs ga{d_jobs, d_items + g.first, g.n};
        void* args[] = {(void*)&ga};
        e = hipLaunchKernel(g.fn, dim3((g.n + g.per_wg - 1) / g.per_wg), dim3(g.threads), args, (size_t)g.lds,
                            sl.stream);
      }
      if (e != hipSuccess) return e;
      gi = end;
    }
    if (P.pn == 0) continue;
    // One persistent kernel over the phase's plain-code requests.
    const int waves = s->cfg.waves_per_cu > 0 ? s->cfg.waves_per_cu : 8;
    int grid = s->cus * waves;
    // Small batches: one item per pop, so that every item has a wave of its
    // own (their tiles are latency-bound walks over the strips).
    const uint32_t chunk = P.pn <= (uint32_t)grid * 2 ? 1u : 4u;
    BatchArgs a{d_jobs, d_items + P.pfirst, P.pn, chunk, d_counter, sl.counter};
    const int need = (int)((P.pn + a.chunk - 1) / a.chunk);
    if (need < grid) grid = std::max(1, need);
    e = batch_launch(a, grid, max_p, sl.stream);
    if (e != hipSuccess) return e;
    sl.counter = batch_counter_after(sl.counter, a.nitems, a.chunk, (uint32_t)grid);
  }
  return hipEventRecord(sl.done, sl.stream);
}

// Builds and launches one admitted batch (its slot busy, not launched).
// Called with the lock held; drops it while it works and returns with it
// held, the slot launched, or its requests failed and the slot free again.
void launch_batch(raid6c_server* s, Slot& sl, std::unique_lock<std::mutex>& lk) {
  const uint64_t launch0 = s->now_ns();
  lk.unlock();
  hipError_t e = hipSuccess;
  bool grew = false;
  if (!s->cfg.plain && !grow_slot(sl, sl.reqs.size(), sl.items, &grew)) e = hipErrorOutOfMemory;
  sl.launch_ns = s->now_ns();
  if (e == hipSuccess) e = launch_slot(s, sl);
  lk.lock();
  s->stats.launch_ns += s->now_ns() - launch0;
  if (grew) s->stats.table_grows++;
  if (e == hipSuccess) {
    sl.launched = true;
    s->cv_done.notify_all();
    return;
  }
  s->thread_error = RAID6C_E_HIP;
  // Fail the batch's requests so callers are not left waiting.
  const uint64_t t = s->now_ns();
  for (const InFlight& f : sl.reqs) {
    f.stripe->refs--;
    if (f.req.kind == RAID6C_REQ_WRITE) {
      f.stripe->failed = true;
      f.stripe->writer = nullptr;
      release_waiters(s, f.stripe);
    }
    complete_one(s, f.req, f.arrival_ns, f.index, RAID6C_ST_INVALID, t, t, 0);
  }
  sl.reqs.clear();
  sl.busy = false;
  s->cv_done.notify_all();
  s->cv_sched.notify_all();
}

void scheduler_loop(raid6c_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    Slot* free_slot = nullptr;
    for (Slot& sl : s->slots)
      if (!sl.busy) {
        free_slot = &sl;
        break;
      }
    if (s->stopping && s->pending.empty() && s->parked == 0) return;
    if (free_slot == nullptr || s->pending.empty()) {
      s->cv_sched.wait(lk);
      continue;
    }
    // Admit requests in arrival order.  A read of a stripe written in this
    // batch runs in its second launch phase; a read of a stripe whose write
    // is in another batch in flight is parked on the stripe until that write
    // completes; a write that must wait for room, and reads of it, are
    // skipped in this pass.  Later requests may pass them.
    Slot& sl = *free_slot;
    sl.reqs.clear();
    const uint64_t admit0 = s->now_ns();
    // When no batch is in flight the GPU is idle: a smaller first batch
    // reaches it sooner, and the next ones are formed while it runs.
    bool idle = true;
    for (const Slot& o : s->slots) idle &= !o.busy;
    size_t max_batch = s->cfg.plain ? 1 : (size_t)std::max(1, s->cfg.max_batch);
    if (idle) max_batch = std::min(max_batch, kIdleBatch);
    size_t items = 0;
    std::unordered_set<uint64_t> waiting_writes;  // skipped writes: reads of them wait too
    for (auto it = s->pending.begin(); it != s->pending.end() && sl.reqs.size() < max_batch;) {
      const raid6c_request& r = it->req;
      int status = check_request(r);
      Resident* st = nullptr;
      bool wait = false;
      if (status == RAID6C_ST_OK && r.kind == RAID6C_REQ_READ && waiting_writes.count(r.stripe_id)) {
        ++it;
        continue;
      }
      if (status == RAID6C_ST_OK && r.kind == RAID6C_REQ_WRITE) {
        if (s->index.find(r.stripe_id) != nullptr) {
          status = RAID6C_ST_DUPLICATE;
        } else {
          bool never = false;
          st = place(s, r, &never);
          if (never) status = RAID6C_ST_TOO_LARGE;
          else if (st == nullptr) wait = true;
        }
      } else if (status == RAID6C_ST_OK) {
        st = s->index.find(r.stripe_id);
        if (st == nullptr) {
          status = RAID6C_ST_NOT_RESIDENT;
        } else {
          if (st->failed || classify(st->k, r.e0, r.e1).op == OP_BAD || r.dst == nullptr ||
              ((uintptr_t)r.dst & 15u) != 0) {
            status = RAID6C_ST_INVALID;
            st = nullptr;
          } else if (!st->ready && st->writer != &sl) {
            st->waiters.push_back(*it);
            s->parked++;
            it = s->pending.erase(it);
            continue;
          }
        }
      }
      if (wait) {
        if (r.kind == RAID6C_REQ_WRITE) waiting_writes.insert(r.stripe_id);
        ++it;
        continue;
      }
      if (status != RAID6C_ST_OK) {
        const uint64_t t = s->now_ns();
        complete_one(s, r, it->arrival_ns, it->index, status, t, t, 0);
        it = s->pending.erase(it);
        s->cv_done.notify_all();
        continue;
      }
      st->refs++;
      int phase = 0;
      if (r.kind == RAID6C_REQ_WRITE) st->writer = &sl;
      else if (!st->ready) phase = 1;   // written in this batch
      sl.reqs.push_back(InFlight{r, it->arrival_ns, it->index, st, phase});
      items += (st->row_bytes + kBatchTileBytes - 1) / kBatchTileBytes;
      it = s->pending.erase(it);
    }
    if (sl.reqs.empty()) {
      // Everything pending waits on in-flight work.
      s->cv_sched.wait(lk);
      continue;
    }
    sl.busy = true;
    sl.items = items;
    s->stats.batches++;
    s->stats.admit_ns += s->now_ns() - admit0;
    launch_batch(s, sl, lk);
  }
}

void completer_loop(raid6c_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    bool any_busy = false, progressed = false;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->stopping && s->outstanding == 0 && s->pending.empty()) {
        bool idle = true;
        for (Slot& sl : s->slots) idle &= !sl.busy;
        if (idle) return;
      }
    }
    for (Slot& sl : s->slots) {
      bool busy;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        busy = sl.busy && sl.launched;
      }
      if (!busy) continue;
      any_busy = true;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) continue;
      progressed = true;
      const uint64_t t = s->now_ns();
      std::lock_guard<std::mutex> lk(s->mu);
      const int n = (int)sl.reqs.size();
      for (const InFlight& f : sl.reqs) {
        if (f.req.kind == RAID6C_REQ_WRITE) {
          f.stripe->ready = q == hipSuccess;
          f.stripe->failed = q != hipSuccess;
          f.stripe->writer = nullptr;
          release_waiters(s, f.stripe);
        }
        f.stripe->refs--;
        const uint64_t user = (uint64_t)f.stripe->k * (f.stripe->p - 1) * f.stripe->row_bytes;
        complete_one(s, f.req, f.arrival_ns, f.index, q == hipSuccess ? RAID6C_ST_OK : RAID6C_ST_INVALID,
                     sl.launch_ns, t, n, user);
      }
      if (q != hipSuccess) s->thread_error = RAID6C_E_HIP;
      sl.reqs.clear();
      sl.launch_ns = 0;
      sl.launched = false;
      sl.busy = false;
      s->cv_sched.notify_all();
      s->cv_done.notify_all();
    }
    if (!any_busy) {
      // Woken by a launch (or a stop); the timeout is a safety net.
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_done.wait_for(lk, std::chrono::microseconds(200));
    } else if (!progressed) {
      std::this_thread::yield();
    }
  }
}

}  // namespace

extern "C" {

int raid6c_server_create(const raid6c_server_config* cfg, raid6c_server** out) {
  if (cfg == nullptr || out == nullptr) return fail(RAID6C_E_ARG, "NULL argument");
  *out = nullptr;
  if (cfg->store_bytes < 4096 || cfg->max_inflight < 1 || cfg->max_inflight > 64 || cfg->max_batch < 1 ||
      cfg->max_batch > 65536 || cfg->waves_per_cu < 0 || cfg->waves_per_cu > 32 ||
      (cfg->persistent != 0 && cfg->persistent != 1))
    return fail(RAID6C_E_ARG, "invalid server configuration");
  raid6c_server* s = new (std::nothrow) raid6c_server();
  if (s == nullptr) return fail(RAID6C_E_NOMEM, "out of host memory");
  s->cfg = *cfg;
  (void)hipGetDevice(&s->device);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device) == hipSuccess && cus > 0)
    s->cus = cus;
  const hipError_t me = hipMalloc((void**)&s->store, cfg->store_bytes);
  if (me != hipSuccess) {
    delete s;
    return fail(RAID6C_E_NOMEM, "cannot allocate a %llu-byte stripe store: %s", (unsigned long long)cfg->store_bytes,
                hipGetErrorString(me));
  }
  s->slots.resize((size_t)cfg->max_inflight);
  // Stripe records for the first few thousand writes, touched now rather
  // than on the first burst.
  for (int i = 0; i < 4096; ++i) {
    s->pool.emplace_back();
    s->free_res.push_back(&s->pool.back());
  }
  hipError_t e = hipSuccess;
  if (cfg->plain) e = hipStreamCreateWithFlags(&s->plain_stream, hipStreamNonBlocking);
  for (Slot& sl : s->slots) {
    if (e != hipSuccess) break;
    if (cfg->plain) sl.stream = s->plain_stream;
    else e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    // Tables for max_batch requests of up to 64 column tiles each (rows up to
    // 16 KiB), at most 4 MiB per slot; larger batches grow them.
    if (e == hipSuccess && !cfg->plain) {
      const size_t jobs = (size_t)cfg->max_batch;
      const size_t items = std::min(jobs * 64, ((size_t)4 << 20) / sizeof(BatchItem));
      if (!grow_slot(sl, jobs, items)) e = hipErrorOutOfMemory;
    }
  }
  if (e != hipSuccess) {
    raid6c_server_destroy(s);
    return fail(RAID6C_E_HIP, "stream or event creation failed: %s", hipGetErrorString(e));
  }
  s->scheduler = std::thread(scheduler_loop, s);
  s->completer = std::thread(completer_loop, s);
  *out = s;
  return RAID6C_OK;
}

int raid6c_server_submit(raid6c_server* s, const raid6c_request* reqs, size_t n) {
  if (s == nullptr || (reqs == nullptr && n != 0)) return fail(RAID6C_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->replay_out != nullptr) return fail(RAID6C_E_STATE, "a replay is running");
  const uint64_t t = s->now_ns();
  for (size_t i = 0; i < n; ++i) s->pending.push_back(Pending{reqs[i], t, SIZE_MAX});
  s->outstanding += n;
  s->stats.submitted += n;
  s->cv_sched.notify_all();
  return RAID6C_OK;
}

int raid6c_server_poll(raid6c_server* s, raid6c_completion* out, size_t cap, size_t* n) {
  if (s == nullptr || n == nullptr || (out == nullptr && cap != 0)) return fail(RAID6C_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  size_t m = 0;
  while (m < cap && !s->done.empty()) {
    out[m++] = s->done.front();
    s->done.pop_front();
  }
  *n = m;
  return RAID6C_OK;
}

int raid6c_server_wait_idle(raid6c_server* s) {
  if (s == nullptr) return fail(RAID6C_E_ARG, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->outstanding == 0; });
  return s->thread_error;
}

int raid6c_server_replay(raid6c_server* s, const raid6c_request* reqs, const double* arrival_s, size_t n,
                         raid6c_completion* out) {
  if (s == nullptr || ((reqs == nullptr || arrival_s == nullptr || out == nullptr) && n != 0))
    return fail(RAID6C_E_ARG, "NULL argument");
  for (size_t i = 1; i < n; ++i)
    if (arrival_s[i] < arrival_s[i - 1]) return fail(RAID6C_E_ARG, "arrival times must not decrease");
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->outstanding == 0; });
    if (s->replay_out != nullptr) return fail(RAID6C_E_STATE, "a replay is running");
    s->replay_out = out;
  }
  // Open loop: request i is submitted at start + arrival_s[i], whatever the
  // state of earlier requests; its latency counts from that scheduled time.
  // Every request that is due when the loop looks is submitted in one
  // critical section (all of them at once when the arrival times are 0).
  const uint64_t start = s->now_ns() + 1000000;  // 1 ms to get going
  auto due_at = [&](size_t i) { return start + (uint64_t)(arrival_s[i] * 1e9); };
  for (size_t i = 0; i < n;) {
    const uint64_t due = due_at(i);
    uint64_t now = s->now_ns();
    while (now < due) {
      const uint64_t left = due - now;
      if (left > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(left - 100000));
      now = s->now_ns();
    }
    // At most 256 per critical section, so that the scheduler can start on
    // a burst while the rest of it is still being submitted.
    std::lock_guard<std::mutex> lk(s->mu);
    for (size_t m = 0; i < n && m < 256 && due_at(i) <= now; ++i, ++m) {
      s->pending.push_back(Pending{reqs[i], due_at(i), i});
      s->outstanding++;
      s->stats.submitted++;
    }
    s->cv_sched.notify_all();
  }
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->outstanding == 0; });
  s->replay_out = nullptr;
  return s->thread_error;
}

int raid6c_server_stripe(raid6c_server* s, uint64_t stripe_id, void** base, uint64_t* strip_stride) {
  if (s == nullptr || base == nullptr || strip_stride == nullptr) return fail(RAID6C_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  const Resident* f = s->index.find(stripe_id);
  if (f == nullptr) return fail(RAID6C_E_ARG, "stripe %llu is not resident", (unsigned long long)stripe_id);
  *base = s->store + f->off;
  *strip_stride = (uint64_t)(f->p - 1) * f->row_bytes;
  return RAID6C_OK;
}

int raid6c_server_get_stats(raid6c_server* s, raid6c_server_stats* out) {
  if (s == nullptr || out == nullptr) return fail(RAID6C_E_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->resident = s->fifo.size();
  uint64_t used = 0;
  for (const Resident* r : s->fifo) used += r->bytes;
  out->store_used = used;
  return RAID6C_OK;
}

int raid6c_server_destroy(raid6c_server* s) {
  if (s == nullptr) return RAID6C_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
    s->cv_sched.notify_all();
    s->cv_done.notify_all();
  }
  if (s->scheduler.joinable()) s->scheduler.join();
  if (s->completer.joinable()) s->completer.join();
  for (Slot& sl : s->slots) {
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream && sl.stream != s->plain_stream) (void)hipStreamDestroy(sl.stream);
    if (sl.h_buf) (void)hipHostFree(sl.h_buf);
    if (sl.d_mem) (void)hipFree(sl.d_mem);
    for (uint8_t* h : sl.retired_h) (void)hipHostFree(h);
    for (uint8_t* d : sl.retired_d) (void)hipFree(d);
  }
  if (s->plain_stream) (void)hipStreamDestroy(s->plain_stream);
  if (s->store) (void)hipFree(s->store);
  delete s;
  return RAID6C_OK;
}

}  // extern "C"
