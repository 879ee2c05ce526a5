// raid6c_internal.h -- types shared by the host API and the kernels of libraid6c.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

struct raid6c_job;  // include/raid6c.h

namespace raid6c {

// Largest prime built into the GPU path (odd primes 3..61).
constexpr int kMaxPrime = 61;
// Up to 2p-1 data strips with the extended Q parity (Section 3.3), + P + Q.
constexpr int kMaxData = 2 * kMaxPrime - 1;
constexpr int kMaxStrips = kMaxData + 2;

// Cases of Lemma 3.1.2 (plus the single erasures and plain encode).
enum : int {
  OP_PQ = 0,   // encode / P and Q erased: recompute both
  OP_P = 1,    // P alone erased
  OP_Q = 2,    // Q alone erased
  OP_D = 3,    // one data strip x erased
  OP_DP = 4,   // data x and P
  OP_DQ = 5,   // data x and Q
  OP_DD = 6,   // data x < y
  OP_BAD = 7,  // invalid erasure entry
};

struct Case {
  int op;
  int x;
  int y;
};

// Classify an erasure entry (e1 = -1: single).  Valid indices are 0..k+1.
__host__ __device__ inline Case classify(int k, int e0, int e1) {
  Case c{OP_BAD, -1, -1};
  const int n = k + 2;
  if (e0 < 0 || e0 >= n) return c;
  if (e1 == -1) {
    if (e0 < k) c = Case{OP_D, e0, -1};
    else if (e0 == k) c = Case{OP_P, -1, -1};
    else c = Case{OP_Q, -1, -1};
    return c;
  }
  if (e1 < 0 || e1 >= n || e1 == e0) return c;
  const int lo = e0 < e1 ? e0 : e1;
  const int hi = e0 < e1 ? e1 : e0;
  if (lo == k) c = Case{OP_PQ, -1, -1};
  else if (hi == k) c = Case{OP_DP, lo, -1};
  else if (hi == k + 1) c = Case{OP_DQ, lo, -1};
  else c = Case{OP_DD, lo, hi};
  return c;
}

// Kernel arguments of the Z_p kernels (passed by value).
struct ZpArgs {
  uint8_t* strip[kMaxStrips];  // strip j of stripe 0 (j = 0..k+1)
  uint64_t stripe_stride;      // bytes between consecutive stripes
  uint64_t row_bytes;          // W
  uint32_t nstripes;
  uint32_t tiles;              // column tiles per row
  int32_t k;
  int32_t e0, e1;              // uniform erasures, used when `erasures` is NULL
  const int32_t* erasures;     // per-stripe pairs (device), or NULL
  int32_t* bad_count;          // device counter of rejected stripes, or NULL
  const uint8_t* src_base;     // write path: data strip j of stripe s is read from
                               // src_base + s*src_stripe_stride + j*src_strip_stride
  uint64_t src_strip_stride;   // and copied to strip j; NULL = encode in place
  uint64_t src_stripe_stride;
  int32_t kind;                // ZpKind of the launch (set by the launcher)
  int32_t shared_lines;        // some row does not start on a 128-byte line (set by the launcher)
  int32_t xcd_order;           // XCD-chunked work-group order (set by the launcher)
  uint32_t stripe_mult;        // 0, or work-group order 2: stripe s -> s*stripe_mult mod nstripes
};

// Launch configuration of a Z_p kernel.
struct ZpConfig {
  int vec;        // dwords per thread and row: 1, 2 or 4
  int unroll;     // data strips whose loads are issued together: 1, 2 or 4
  int threads;    // work-group size: 64, 128 or 256
  int split = 1;  // waves sharing one column tile (1, 2, 4); threads = 64*split when > 1
  int order = 0;  // 1: XCD-chunked work-group order (always taken when rows are off 128-byte lines);
                  // 2: stripes spread over the launch (a fixed permutation of the stripe index)
};

enum ZpKind : int { KIND_ENCODE = 0, KIND_RECOVER = 1 };

// Per-prime launchers, six translation units per prime (zp_kernels.hip).
// Return hipSuccess or the launch error (hipErrorInvalidValue for a
// configuration that is not built).
typedef hipError_t (*ZpLauncher)(ZpKind kind, const ZpConfig& cfg, const ZpArgs& a,
                                 uint32_t grid, hipStream_t stream);

struct BatchJob;
struct BatchItem;
// A plan's jobs of one prime run as one grid of the per-prime job-list
// kernel (zp_kernels.hip, variant 3).
struct GroupArgs {
  const BatchJob* jobs;
  const BatchItem* items;    // this group's items (tiles of 64 lanes x group_vec dwords)
  uint32_t nitems;
};
struct ZpPrimeEntry {
  int p;
  ZpLauncher launch;       // plain code, k <= p, and every split-K configuration (any k)
  ZpLauncher launch_ext;   // extended Q parity, p < k <= 2p-1
  int vec_mask;        // bit v set when vec = v is instantiated (bits 1, 2, 4)
  int unroll_mask[5];  // per vec: bit u set when (vec, unroll = u) is instantiated
  int split_mask[5];   // per vec: bit s set when split = s (2, 4) is built
  // Job-list kernel, __global__ void(GroupArgs), and its launch shape: items
  // are tiles of 64 lanes x group_vec dwords; a work-group of group_threads
  // threads takes group_per_wg consecutive items (4: one per wave; 1: its
  // waves split the strips of one item) and group_lds bytes of dynamic LDS.
  const void* group_kernel;
  int group_vec;
  int group_per_wg;
  int group_threads;
  int group_lds;
  // The same kernel for jobs with the extended Q parity (k > p): same
  // launch shape; group_ext_vec equals group_vec.
  const void* group_ext_kernel;
  int group_ext_vec;
  // The job-list kernel for batches too small to fill the GPU (the server's):
  // set for the latency of one tile.  Tiles of 64 lanes x group_lat_vec
  // dwords, one per work-group of group_lat_threads threads (its waves split
  // the strips), group_lat_lds bytes of dynamic LDS.
  const void* group_lat_kernel;
  int group_lat_vec;
  int group_lat_threads;
  int group_lat_lds;

  // Job-list kernel for jobs with k data strips.
  const void* group_fn(int k) const { return k > p ? group_ext_kernel : group_kernel; }

  bool has(int vec, int unroll) const {
    return (vec == 1 || vec == 2 || vec == 4) && (vec_mask & vec) &&
           (unroll == 1 || unroll == 2 || unroll == 4) && (unroll_mask[vec] & unroll);
  }
  bool has(const ZpConfig& c) const {
    if (!has(c.vec, c.unroll) || c.order < 0 || c.order > 2) return false;
    if (c.split == 1) return c.threads == 64 || c.threads == 128 || c.threads == 256;
    return (c.split == 2 || c.split == 4) && (split_mask[c.vec] & c.split) && c.threads == 64 * c.split;
  }
};

const ZpPrimeEntry* zp_prime_entry(int p);  // NULL when p is not built

// Persistent mixed-geometry kernel (batch.hip), shared by plans and the
// request server.
struct BatchJob {
  uint8_t* base;          // strip 0 of the stripe
  uint64_t strip_stride;  // bytes between its strips
  uint8_t* out0;          // where erased strip x0 is written (in place: base + x0*stride)
  uint8_t* out1;
  const uint8_t* src;     // write from a payload: data strip j at src + j*src_stride; else NULL
  uint64_t src_stride;
  uint32_t row_bytes;
  int16_t p, k;
  int16_t op, x, y;       // Case
  int16_t e0, e1;         // the strips redirected to out0 / out1 (-1: none)
  int16_t pad;
};

struct BatchItem {
  uint32_t job;
  uint32_t col;  // byte offset of the 256-byte tile within a row
};

struct BatchArgs {
  const BatchJob* jobs;
  const BatchItem* items;
  uint32_t nitems;
  uint32_t chunk;       // items taken per counter increment
  uint64_t* counter;    // work counter: the run takes values base, base+chunk, ...
  uint64_t base;
};

// Value of the counter after a run of `nitems` items with `grid` work-groups
// started at `base`: every work-group stops at its first pop past the end,
// so the run takes exactly ceil(nitems/chunk) + grid increments of `chunk`.
inline uint64_t batch_counter_after(uint64_t base, uint32_t nitems, uint32_t chunk, uint32_t grid) {
  return base + ((uint64_t)(nitems + chunk - 1) / chunk + grid) * chunk;
}

constexpr int kBatchTileBytes = 256;  // 64 lanes x one dword

// Enqueue the persistent kernel on `stream` (grid work-groups of one wave,
// LDS for primes up to max_p); the counter must hold a.base.
hipError_t batch_launch(const BatchArgs& a, int grid, int max_p, hipStream_t stream);

// Checks of one job of a job list (batch.hip): *out receives its case.
// Returns RAID6C_OK or an error code (the message names job i).
int check_job(const ::raid6c_job& J, size_t i, Case* out);
// The device-side description of a checked job (in place: no redirected
// strips, no payload source).
BatchJob make_batch_job(const ::raid6c_job& J, const Case& cs);

// Kernel functions, for graph nodes.
const void* batch_kernel_fn();
const void* batch_reset_fn();

// Reed-Solomon GF(256) comparison kernel (rs_kernels.hip).
struct RsArgs {
  uint8_t* base;
  uint64_t strip_stride;
  uint64_t stripe_stride;
  uint64_t strip_bytes;
  uint32_t nstripes;
  uint32_t tiles;
  int32_t k;
  const int32_t* erasures;  // per-stripe pairs (device), or NULL: encode P and Q
  int32_t* bad_count;       // device counter of rejected entries, or NULL
};
hipError_t rs_launch(const RsArgs& a, int vec, int unroll, int threads, uint32_t grid, hipStream_t stream);

// Small-write kernels (update.hip).
struct UpdArgs {
  uint8_t* base;               // strided stripes (strip j of stripe s at base + s*stripe_stride +
  uint64_t strip_stride;       // j*strip_stride), or NULL for one stripe given by pd, pp, pq
  uint64_t stripe_stride;
  uint8_t* pd;                 // one stripe: data strip t, P and Q
  uint8_t* pp;
  uint8_t* pq;
  const uint8_t* src;          // new data strip of stripe s at src + s*src_stride
  uint64_t src_stride;
  const int32_t* targets;      // per-stripe data strip index (device), or NULL: `t` for all
  int32_t* bad_count;          // device counter of rejected entries, or NULL
  uint64_t row_bytes;
  uint32_t nstripes;
  uint32_t tiles;
  int32_t t;
  int32_t k;
};
// shared_lines: rows not all on 128-byte lines (ordinary-policy loads,
// XCD-chunked work-group order).
hipError_t update_launch(const UpdArgs& a, int p, int vec, int threads, uint32_t grid, bool shared_lines,
                         hipStream_t stream);

// Horizontal Z_17 layout <-> vertical strips (layout.hip): count strips of
// 8*row_bytes 16-bit words <-> count strips of 16 rows of row_bytes bytes.
hipError_t z17_launch(bool to_vertical, const void* in, void* out, uint64_t row_bytes, uint64_t count,
                      hipStream_t stream);

}  // namespace raid6c
