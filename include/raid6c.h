/*
 * raid6c.h -- cyclic-group RAID-6 (Z_p-RAID) on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libraid6c.so.  The code is the one of Jackson, Rumynin and
 * Zaboronski, "An approach to RAID-6 based on cyclic groups":
 *
 *   P = D_0 + D_1 + ... + D_{k-1}
 *   Q = D_0 + g D_1 + ... + g^{k-1} D_{k-1}
 *
 * in the ring R_p = F2[x]/(1 + x + ... + x^{p-1}), g = x acting as the
 * Sylvester matrix S_p (Corollary 3.2.4 with Lemma 3.4.1), p an odd prime,
 * 1 <= k <= p data strips.  Any one or two strips of a stripe can be rebuilt
 * from the others (Lemma 3.1.2).
 *
 * Extended Q parity (Section 3.3, eq. qext): for primes that satisfy
 * Theorem 3.3.3 (all supported primes except the Mersenne primes 3, 7, 31),
 * up to 2p-1 data strips, strip t >= p entering Q with 1 + g^{t-p+1}:
 *
 *   Q = sum_{t<p} g^t D_t + sum_{t>=p} (1 + g^{t-p+1}) D_t
 *
 * For k <= p this is the code above.  The single-stripe and strided entry
 * points, writes and degraded reads accept k up to raid6c_max_data_strips(p);
 * plans and the request server run k <= p only.
 *
 * Layout.  A strip is p-1 rows of row_bytes bytes, row r at byte offset
 * r*row_bytes; bit b of byte j of row r is the coefficient of x^r of lane
 * (j, b), so every lane is an independent ring element.  A stripe is k data
 * strips (indices 0..k-1), then P (index k), then Q (index k+1).
 *
 * Conventions for every entry point below:
 *  - All buffers are device memory owned by the caller; the library never
 *    keeps a pointer after the call returns (plans excepted, see there).
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *    is complete when the stream is; the calls do not synchronise.
 *  - row_bytes must be a positive multiple of 16 and every strip pointer
 *    16-byte aligned (the kernels move 16-, 8- or 4-byte vectors).
 *  - Strips of one stripe must not overlap; different stripes must not
 *    overlap in the strips a call writes.
 *  - Arguments are checked before any device work: on an error nothing is
 *    enqueued and nothing is written.  Return values: RAID6C_OK (0) or a
 *    negative RAID6C_E_* code; raid6c_last_error() gives a message.
 *  - Arithmetic is exact (XOR only); results are bit-exact.
 *  - The calls are reentrant; they keep no state between calls.
 */
#ifndef RAID6C_H
#define RAID6C_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RAID6C_OK              0
#define RAID6C_E_ARG          (-1) /* invalid argument (bad p, k, index, size, alignment) */
#define RAID6C_E_UNSUPPORTED  (-2) /* valid for the code but not built into the GPU path (p too large) */
#define RAID6C_E_HIP          (-3) /* HIP runtime or launch failure */
#define RAID6C_E_NOMEM        (-4) /* device or host allocation failed (plans, servers) */
#define RAID6C_E_STATE        (-5) /* call not valid in the object's current state */

/* Largest prime p the GPU kernels are built for; every odd prime up to it is
 * supported.  Primes above it return RAID6C_E_UNSUPPORTED. */
int raid6c_max_prime(void);

/* 1 when p is an odd prime <= raid6c_max_prime(), else 0. */
int raid6c_is_supported_prime(int p);

/* Largest number of data strips k for prime p: 2p-1 when p satisfies
 * condition (3) of Theorem 3.3.3 (X^p + 1 and X^m + X + 1 coprime over F2
 * for 0 < m < p), so that the extended Q parity exists; p otherwise.
 * Errors: RAID6C_E_ARG if p is not an odd prime; RAID6C_E_UNSUPPORTED if
 * p > raid6c_max_prime(). */
int raid6c_max_data_strips(int p);

/* Static text for a RAID6C_* code. */
const char* raid6c_strerror(int code);

/* Message of the last failed call on this host thread ("" if none). */
const char* raid6c_last_error(void);

/* ------------------------------------------------------------------------
 * Single stripe
 * ------------------------------------------------------------------------ */

/* Encode one stripe: P = sum_t D_t, Q = sum_t g^t D_t (Corollary 3.2.4; the
 * 0-based indexing of the Reed-Solomon parity of Section 4.1).
 *   data : host array of k device pointers, data[t] = strip D_t (read only)
 *   P, Q : device strips written with the parities
 * With k > p the parity is the extended one (eq. qext).
 * Errors: RAID6C_E_ARG if p is not an odd prime, k not in
 * [1, raid6c_max_data_strips(p)], row_bytes not a positive multiple of 16,
 * or a pointer NULL or misaligned;
 * RAID6C_E_UNSUPPORTED if p > raid6c_max_prime(). */
int raid6c_encode(int p, int k, size_t row_bytes, const void* const* data,
                  void* P, void* Q, void* stream);

/* Rebuild one erased strip e (0..k+1) in place from the k+1 others.
 * Data strip: D_e = P + sum_{t != e} D_t (RAID-5 parity, Section 1); P or Q:
 * recomputed from the data (first / second parity equation).
 *   strips : host array of k+2 device pointers (D_0..D_{k-1}, P, Q); only
 *            strips[e] is written, its input contents are ignored.
 * Errors: as raid6c_encode, plus RAID6C_E_ARG if e is out of range. */
int raid6c_recover_1(int p, int k, size_t row_bytes, void* const* strips,
                     int e, void* stream);

/* Rebuild two erased strips e0 != e1 (any order, 0..k+1) in place
 * (Lemma 3.1.2; the two-data case as in Sections 4.3 and 4.6):
 *   P+Q       : both recomputed from the data;
 *   D_x + P   : D_x = g^{p-x}(Q + sum_{t != x} g^t D_t), then P;
 *   D_x + Q   : D_x = P + sum_{t != x} D_t, then Q;
 *   D_x + D_y : (x < y, z = y-x) dP = P + P_xy, dQ = Q + Q_xy,
 *               D_y = (1+g^z)^{-1}(dP + g^{p-x} dQ), D_x = D_y + dP.
 *   strips : host array of k+2 device pointers; only the two erased strips
 *            are written, their input contents are ignored.
 * Errors: as raid6c_recover_1, plus RAID6C_E_ARG if e0 == e1. */
int raid6c_recover_2(int p, int k, size_t row_bytes, void* const* strips,
                     int e0, int e1, void* stream);

/* ------------------------------------------------------------------------
 * Many stripes of one geometry in one launch (strided layout)
 *
 * Strip j of stripe s starts at base + s*stripe_stride + j*strip_stride,
 * j = 0..k+1.  Both strides are byte counts, multiples of 16, with
 * strip_stride >= (p-1)*row_bytes and, when nstripes > 1,
 * stripe_stride >= (k+2)*strip_stride (strips never overlap).  nstripes = 0
 * is a valid empty call.
 * ------------------------------------------------------------------------ */

/* Encode nstripes stripes: writes the P and Q strips of each (same math as
 * raid6c_encode).  Errors: as raid6c_encode, plus RAID6C_E_ARG for strides
 * that are misaligned or let strips overlap. */
int raid6c_encode_n(int p, int k, size_t row_bytes, void* base,
                    size_t strip_stride, size_t stripe_stride, size_t nstripes,
                    void* stream);

/* Rebuild, per stripe, the one or two strips named by
 * erasures[2s], erasures[2s+1] (device int32 array of 2*nstripes entries;
 * erasures[2s+1] = -1 means a single erasure).  Same math as
 * raid6c_recover_1 / raid6c_recover_2; only erased strips are written.
 * The erasure array lives on the device, so it is checked by the kernel: a
 * stripe whose entries are invalid (out of range, equal, or a first entry
 * of -1) is left untouched and, when bad_count (device int32, may be NULL)
 * is given, counted into *bad_count with an atomic add.
 * Errors: as raid6c_encode_n, plus RAID6C_E_ARG if erasures is NULL or
 * misaligned. */
int raid6c_recover_n(int p, int k, size_t row_bytes, void* base,
                     size_t strip_stride, size_t stripe_stride, size_t nstripes,
                     const int32_t* erasures, int32_t* bad_count, void* stream);

/* ------------------------------------------------------------------------
 * Write path and degraded read of one stripe
 * ------------------------------------------------------------------------ */

/* Write a stripe from a payload: data strip t is read from
 * src + t*src_strip_stride, stored to strips[t], and P and Q (strips[k],
 * strips[k+1]) are computed from it in the same pass (Corollary 3.2.4).
 *   src    : device payload, k strips of (p-1)*row_bytes bytes (read only);
 *            src_strip_stride a multiple of 16, >= (p-1)*row_bytes
 *   strips : host array of k+2 device pointers (written)
 * The payload must not overlap the stripe.  Errors: as raid6c_encode, plus
 * RAID6C_E_ARG for a NULL or misaligned source or a bad stride. */
int raid6c_write(int p, int k, size_t row_bytes, const void* src, size_t src_strip_stride,
                 void* const* strips, void* stream);

/* Degraded read: rebuild the erased strip(s) e0 (and e1 unless -1) of a
 * stripe into `out` without writing the stripe (Lemma 3.1.2 as in
 * raid6c_recover_1 / raid6c_recover_2).  `out` receives the rebuilt strips
 * in ascending strip order, each (p-1)*row_bytes bytes, contiguous.
 *   strips : host array of k+2 device pointers; only the surviving strips
 *            are read, the erased entries may be NULL.
 * Errors: as raid6c_recover_2 (or raid6c_recover_1 when e1 = -1), plus
 * RAID6C_E_ARG for a NULL or misaligned `out` or one overlapping a strip. */
int raid6c_read_degraded(int p, int k, size_t row_bytes, const void* const* strips, int e0, int e1,
                         void* out, void* stream);

/* ------------------------------------------------------------------------
 * Small writes
 * ------------------------------------------------------------------------ */

/* Replace data strip t of one stripe with new_strip and update P and Q from
 * the change alone: the parity equations (Corollary 3.2.4) are linear, so
 * with dD = D_t + D_t'
 *   P' = P + dD,   Q' = Q + g_t dD,
 * g_t = g^t, or 1 + g^{t-p+1} for a strip t >= p of the extended Q parity
 * (the Q-parity update that Section 3.4 prices at shifts and XORs).
 * Reads strips[t], new_strip, strips[k], strips[k+1]; writes strips[t]
 * (= new_strip), strips[k], strips[k+1]; no other strip is touched.  The
 * stripe must be consistent before the call for the result to be.
 *   strips    : host array of k+2 device pointers (entries other than t, k,
 *               k+1 are not used and may be NULL)
 *   new_strip : device, (p-1)*row_bytes bytes, must not overlap the strips
 * Errors: as raid6c_encode, plus RAID6C_E_ARG for t not in [0, k) or a NULL,
 * misaligned or overlapping strip. */
int raid6c_update(int p, int k, size_t row_bytes, void* const* strips, int t,
                  const void* new_strip, void* stream);

/* Small writes on nstripes strided stripes: stripe s replaces data strip
 * targets[s] (device int32 array) with the strip at src + s*src_stride,
 * as raid6c_update.  An entry outside [0, k) leaves its stripe untouched and
 * is counted into *bad_count (device int32, may be NULL).  The sources must
 * not overlap the stripes.
 * Errors: as raid6c_encode_n, plus RAID6C_E_ARG for NULL or misaligned
 * targets or src, or src_stride below (p-1)*row_bytes or not a multiple of
 * 16 (when nstripes > 1). */
int raid6c_update_n(int p, int k, size_t row_bytes, void* base,
                    size_t strip_stride, size_t stripe_stride, size_t nstripes,
                    const int32_t* targets, const void* src, size_t src_stride,
                    int32_t* bad_count, void* stream);

/* ------------------------------------------------------------------------
 * The paper's horizontal Z_17 layout
 *
 * Section 4.5 keeps one codeword of R_17 per 16-bit word, bit r being the
 * coefficient of x^r (so that g.x = (x + x) ^ (x < 0 ? 0xffff : 0)).  A
 * horizontal strip of 8*row_bytes words and a vertical strip of 16 rows of
 * row_bytes bytes hold the same codewords when codeword c is lane
 * (byte c/8, bit c%8) of the vertical strip; parity computed in either
 * layout is the same after conversion.
 * ------------------------------------------------------------------------ */

/* Convert `count` consecutive horizontal strips (words + s*8*row_bytes
 * uint16, device) into vertical strips (strips + s*16*row_bytes, row r at
 * r*row_bytes, device).  row_bytes: a positive multiple of 16; buffers
 * 16-byte aligned and not overlapping.  Errors: RAID6C_E_ARG. */
int raid6c_z17_to_vertical(const void* words, size_t row_bytes, size_t count, void* strips, void* stream);

/* The inverse conversion, same layouts and errors. */
int raid6c_z17_to_horizontal(const void* strips, size_t row_bytes, size_t count, void* words, void* stream);

/* ------------------------------------------------------------------------
 * Comparison code: Reed-Solomon RAID-6 over GF(256), polynomial 0x11D
 * ------------------------------------------------------------------------ */

/* Encode nstripes Reed-Solomon stripes (Section 4.1):
 * P = sum_t D_t, Q = sum_t {02}^t D_t bytewise in GF(2)[x]/(x^8+x^4+x^3+x^2+1),
 * Q by Horner's rule with the multiply-by-{02} of Section 4.2.
 * Each strip is strip_bytes bytes (a positive multiple of 16); strip j of
 * stripe s starts at base + s*stripe_stride + j*strip_stride, j = 0..k-1 data,
 * k = P, k+1 = Q.  1 <= k <= 255 (the order of {02}).
 * Errors: RAID6C_E_ARG for k out of range, sizes, strides or alignment. */
int raid6c_rs_encode_n(int k, size_t strip_bytes, void* base,
                       size_t strip_stride, size_t stripe_stride, size_t nstripes,
                       void* stream);

/* Rebuild, per Reed-Solomon stripe, the one or two disks named by
 * erasures[2s], erasures[2s+1] (device int32, 2*nstripes entries; second
 * entry -1 = single erasure; indices 0..k-1 data, k = P, k+1 = Q), by the
 * cases of Lemma 3.1.2 for the cone {g^t}:
 *   data x + P:  D_x = g^{-x} (Q + Q_x), then P;
 *   data x + Q:  D_x = P + P_x, then Q;
 *   data x < y:  D_y = A (P + P_xy) + B (Q + Q_xy), D_x = D_y + P + P_xy with
 *                A = (1 + g^{y-x})^{-1}, B = (g^x + g^y)^{-1} (Sections 4.3-4.4);
 *   P and/or Q alone, one data disk: recomputed / RAID-5 parity.
 * Layout and errors as raid6c_rs_encode_n, plus RAID6C_E_ARG if erasures is
 * NULL or misaligned.  Invalid entries are skipped and counted into
 * *bad_count (device int32, may be NULL), as in raid6c_recover_n; only the
 * erased disks are written. */
int raid6c_rs_recover_n(int k, size_t strip_bytes, void* base,
                        size_t strip_stride, size_t stripe_stride, size_t nstripes,
                        const int32_t* erasures, int32_t* bad_count, void* stream);

/* Fix the launch configuration of the Reed-Solomon kernels for this process
 * (vec dwords per thread: 1, 2, 4; unroll strips loaded together: 1, 4, 8;
 * threads: 64, 128, 256); (0, 0, 0) restores the built-in rule.
 * Errors: RAID6C_E_ARG for a configuration that is not built. */
int raid6c_rs_set_config(int vec, int unroll, int threads);

/* ------------------------------------------------------------------------
 * Plans: many stripes of mixed p, k and row size in one graph launch
 *
 * A plan is built once from a job list and replayed any number of times.
 * Each replay is one HIP graph launch.  With the default (grouped) schedules
 * the graph holds one grid per prime present: a job-list kernel compiled for
 * that prime, whose waves each take one column tile of one stripe.  With the
 * persistent schedule it holds a single persistent kernel for all primes
 * (plus a one-thread kernel that resets its work counter), whose single-wave
 * work-groups take 256-byte column tiles from a device counter.  The
 * per-stripe math is that of raid6c_encode / raid6c_recover_1 /
 * raid6c_recover_2, bit for bit, under every schedule.
 * ------------------------------------------------------------------------ */

#define RAID6C_JOB_ENCODE   0  /* write P and Q from the data strips */
#define RAID6C_JOB_RECOVER  1  /* rebuild strips e0 (and e1, unless -1) */

/* One stripe of a plan: strip j (0..k-1 data, k = P, k+1 = Q) starts at
 * base + j*strip_stride (device memory, 16-byte aligned, strip_stride a
 * multiple of 16 and >= (p-1)*row_bytes).  Strips of different jobs must not
 * share any byte.  e0/e1 are ignored for encode jobs. */
typedef struct raid6c_job {
  int32_t op;
  int32_t p;
  int32_t k;
  int32_t e0;
  int32_t e1;
  uint32_t row_bytes;
  uint64_t strip_stride;
  void* base;
} raid6c_job;

#define RAID6C_ORDER_LARGEST_FIRST 0  /* items of the costliest stripes first */
#define RAID6C_ORDER_BY_PRIME      1  /* grouped by p (largest p first) */
#define RAID6C_ORDER_SUBMITTED     2  /* job order as given */

/* Schedule of a plan.  Changes speed only.
 *  grouped = 1: the jobs of each prime run as one grid of a
 *    job-list kernel compiled for that prime (tiles of 64 lanes x 2 dwords
 *    up to p = 53, x 1 dword above; 4 waves per work-group, one tile each);
 *    the grids are independent nodes of the plan's graph and may run side
 *    by side.  The other fields are kept but unused.
 *  grouped = 2 (the default): the same grids, chained in the graph so that
 *    they run one after another, largest prime first.
 *  grouped = 0: one persistent kernel for all primes; waves_per_cu
 *    persistent work-groups per compute unit take `chunk` 256-byte tiles per
 *    increment of a device counter, in `order`. */
typedef struct raid6c_schedule {
  int32_t waves_per_cu;  /* 1..32 */
  int32_t chunk;         /* 1..1024 */
  int32_t order;         /* RAID6C_ORDER_* */
  int32_t grouped;       /* 0, 1 or 2 */
} raid6c_schedule;

typedef struct raid6c_plan_info {
  uint64_t njobs;
  uint64_t nitems;
  uint64_t bytes_moved;  /* algorithmic HBM bytes per run */
  uint64_t user_bytes;   /* sum of k*(p-1)*row_bytes */
  int32_t max_p;
  int32_t grid;          /* work-groups per run (all grids of a grouped run) */
} raid6c_plan_info;

typedef struct raid6c_plan raid6c_plan;

/* Build a plan for njobs jobs on the current device.  The plan owns device
 * memory for its job and item tables (freed by raid6c_plan_destroy) and keeps
 * the job addresses, which must stay valid while the plan is used.  This call
 * synchronises with the device (uploads).  Errors: RAID6C_E_ARG for an
 * invalid job (its index is in raid6c_last_error()) or overlapping strips,
 * RAID6C_E_UNSUPPORTED for p above raid6c_max_prime(), RAID6C_E_NOMEM,
 * RAID6C_E_HIP.  njobs = 0 gives an empty plan whose runs do nothing. */
int raid6c_plan_create(const raid6c_job* jobs, size_t njobs, raid6c_plan** out);

/* Enqueue one run of the plan on `stream` (a graph launch).  Runs are
 * idempotent: every job rewrites the same bytes.  Runs of one plan on
 * different streams must not overlap in time (they share the work counter).
 * Errors: RAID6C_E_ARG (NULL plan), RAID6C_E_HIP. */
int raid6c_plan_run(raid6c_plan* plan, void* stream);

/* Current schedule / replace it (rebuilds the graph; synchronises).
 * Errors: RAID6C_E_ARG for NULL arguments or an invalid schedule. */
int raid6c_plan_get_schedule(const raid6c_plan* plan, raid6c_schedule* out);
int raid6c_plan_set_schedule(raid6c_plan* plan, const raid6c_schedule* schedule);

/* Sizes of the plan.  Errors: RAID6C_E_ARG for NULL arguments. */
int raid6c_plan_stats(const raid6c_plan* plan, raid6c_plan_info* out);

/* Autotuner: time every candidate schedule (grouped side by side, grouped
 * one after another, and the persistent kernel with waves per CU x chunk x
 * order)
 * over `reps` runs each on `stream`, keep the fastest, and return its mean
 * time per run in *best_ms (may be NULL).  Runs the plan (reps+1) times per
 * candidate, which rewrites the same output bytes.  Synchronises.
 * Errors: RAID6C_E_ARG (NULL plan, reps outside 1..1000), RAID6C_E_HIP. */
int raid6c_plan_autotune(raid6c_plan* plan, void* stream, int reps, float* best_ms);

/* Free the plan and its device memory (NULL is allowed). */
int raid6c_plan_destroy(raid6c_plan* plan);

/* Run every job as its own plain launch (raid6c_encode_n with one stripe,
 * raid6c_recover_1 or raid6c_recover_2), in order, on `stream`: the
 * per-request path that plans replace.  Jobs are checked as by
 * raid6c_plan_create (except for overlap); on an invalid job nothing is
 * launched.  Errors: as raid6c_plan_create. */
int raid6c_run_jobs(const raid6c_job* jobs, size_t njobs, void* stream);

/* Limits of raid6c_run_jobs_noalloc: jobs per call, and column tiles per call
 * (a job has ceil(row_bytes / 512) tiles for p <= 31, ceil(row_bytes / 256)
 * above). */
#define RAID6C_NOALLOC_MAX_JOBS 4096
#define RAID6C_NOALLOC_MAX_ITEMS 262144

/* For callers that cannot allocate (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): the jobs of a job list run as a
 * plan's grouped schedule runs them (one grid of each prime's job-list
 * kernel, on `stream`), with the same results, but nothing is allocated.  The
 * job and item tables are staged in a fixed device array of about 2.3 MiB
 * that the library holds on each GPU it runs on until the process ends, and
 * in a fixed host array.  Jobs are checked as by raid6c_run_jobs (not for
 * overlap: strips of different jobs must not share bytes); on an invalid job,
 * or beyond RAID6C_NOALLOC_MAX_JOBS jobs or RAID6C_NOALLOC_MAX_ITEMS tiles
 * (RAID6C_E_ARG), nothing is launched.  The tables are copied from pageable
 * host memory, which the runtime does synchronously: the call returns after
 * the copy, which waits for the work queued before it on `stream`.  Calls on
 * one stream are therefore ordered; calls on one GPU whose work overlaps
 * (different streams, or host threads that do not wait for each other's
 * work) share the one device array and race.  Errors: as raid6c_run_jobs,
 * RAID6C_E_HIP. */
int raid6c_run_jobs_noalloc(const raid6c_job* jobs, size_t njobs, void* stream);

/* ------------------------------------------------------------------------
 * Request server: continuous batching of writes and degraded reads
 *
 * The server owns a stripe store of `store_bytes` of device memory (its HBM
 * budget), used as a ring in arrival order; a write that needs room evicts
 * the oldest stripes that no admitted request is using, and waits while the
 * oldest one is busy.  A scheduler thread admits pending requests into free
 * slots (up to max_inflight batches on their own streams, max_batch requests
 * each) and launches each batch as one job-list grid per prime (small groups
 * of the primes up to 31 in one grid together), or as one persistent kernel
 * (`persistent`); requests arriving
 * meanwhile go into the next free slot, so batches overlap on the device.  A
 * completion thread reports each request with its arrival, launch and
 * completion times (ns on the server's steady clock).  With `plain` set,
 * every request is one plain launch (raid6c_write / raid6c_read_degraded)
 * on a single stream instead: the per-request path, for comparison.
 * Results are bit-identical either way.
 * ------------------------------------------------------------------------ */

#define RAID6C_REQ_WRITE 0  /* payload -> new resident stripe (data + P + Q) */
#define RAID6C_REQ_READ  1  /* rebuild erased strip(s) of a resident stripe into dst */

#define RAID6C_ST_OK            0
#define RAID6C_ST_NOT_RESIDENT  1  /* read of an unknown or evicted stripe */
#define RAID6C_ST_TOO_LARGE     2  /* stripe larger than the whole store */
#define RAID6C_ST_INVALID       3  /* bad geometry, erasures or buffers */
#define RAID6C_ST_DUPLICATE     4  /* write of a stripe id that is resident */

/* A write gives p, k, row_bytes, a new stripe_id and `src`: the device
 * payload, k strips of (p-1)*row_bytes bytes back to back, which must stay
 * valid until the request completes.  A read gives the stripe_id, the erased
 * strips e0 and e1 (-1 for one) and `dst`: a device buffer, not overlapping
 * the store, that receives the rebuilt strips in ascending strip order.
 * `tag` is returned with the completion. */
typedef struct raid6c_request {
  int32_t kind;
  int32_t p;
  int32_t k;
  int32_t e0;
  int32_t e1;
  uint32_t row_bytes;
  uint64_t stripe_id;
  const void* src;
  void* dst;
  uint64_t tag;
} raid6c_request;

typedef struct raid6c_completion {
  uint64_t tag;
  int32_t status;       /* RAID6C_ST_* */
  int32_t batch_size;   /* requests launched together with this one */
  uint64_t arrival_ns;  /* submission (or scheduled arrival in a replay) */
  uint64_t launch_ns;
  uint64_t complete_ns;
} raid6c_completion;

typedef struct raid6c_server_config {
  uint64_t store_bytes;  /* HBM budget of the stripe store, >= 4096 */
  int32_t max_inflight;  /* batches in flight, 1..64 */
  int32_t max_batch;     /* requests per batch, 1..65536 */
  int32_t plain;         /* 1: one plain launch per request on one stream */
  int32_t waves_per_cu;  /* persistent work-groups per compute unit (0 = 8) */
  int32_t persistent;    /* 0: a batch is one grid of the job-list kernel per prime present
                            (as a plan's grouped schedule); 1: one persistent kernel */
} raid6c_server_config;

typedef struct raid6c_server_stats {
  uint64_t submitted;
  uint64_t completed;
  uint64_t batches;
  uint64_t evictions;
  uint64_t user_bytes;   /* k*(p-1)*row_bytes of every successful request */
  uint64_t resident;     /* stripes in the store */
  uint64_t store_used;   /* bytes they occupy */
  uint64_t table_grows;  /* batches whose slot had to enlarge its job/item tables */
  uint64_t admit_ns;     /* scheduler time spent admitting requests into batches */
  uint64_t launch_ns;    /* scheduler time spent building tables and launching batches */
} raid6c_server_stats;

typedef struct raid6c_server raid6c_server;

/* Create a server on the current device (allocates the store, streams and
 * two host threads).  Errors: RAID6C_E_ARG, RAID6C_E_NOMEM, RAID6C_E_HIP. */
int raid6c_server_create(const raid6c_server_config* cfg, raid6c_server** out);

/* Queue requests (thread-safe); their arrival time is now.  Bad requests
 * complete with a status, not an error.  Errors: RAID6C_E_ARG,
 * RAID6C_E_STATE while a replay runs. */
int raid6c_server_submit(raid6c_server* s, const raid6c_request* reqs, size_t n);

/* Take up to `cap` completions (in completion order); *n receives the count. */
int raid6c_server_poll(raid6c_server* s, raid6c_completion* out, size_t cap, size_t* n);

/* Block until every submitted request has completed.  Returns RAID6C_E_HIP if
 * a launch or kernel failed since the server started. */
int raid6c_server_wait_idle(raid6c_server* s);

/* Open-loop replay: submit request i at (start + arrival_s[i]) seconds, from
 * the calling thread, whatever the state of earlier requests, then wait for
 * all; out[i] receives request i's completion, whose arrival_ns is the
 * scheduled time.  arrival_s must not decrease.  Errors: RAID6C_E_ARG,
 * RAID6C_E_STATE, RAID6C_E_HIP. */
int raid6c_server_replay(raid6c_server* s, const raid6c_request* reqs, const double* arrival_s, size_t n,
                         raid6c_completion* out);

/* Location of a resident stripe: *base receives the device address of its
 * strip 0 and *strip_stride the bytes between strips (valid until the stripe
 * is evicted).  Errors: RAID6C_E_ARG (NULL arguments or not resident). */
int raid6c_server_stripe(raid6c_server* s, uint64_t stripe_id, void** base, uint64_t* strip_stride);

/* Counters of the server so far. */
int raid6c_server_get_stats(raid6c_server* s, raid6c_server_stats* out);

/* Finish every queued request, stop the threads and free the server. */
int raid6c_server_destroy(raid6c_server* s);

/* ------------------------------------------------------------------------
 * Launch configuration (used by the autotuner and by tests)
 *
 * A Z_p kernel launch is configured by `vec`, the dwords each thread moves
 * per row (1, 2 or 4), `unroll`, the number of data strips whose loads are
 * issued together (1, 2 or 4), `threads`, the work-group size (64, 128 or
 * 256), and `split`: 1 = every thread of the work-group owns its own column
 * slice; 2 or 4 = the work-group's `split` waves share one column tile of 64
 * lanes and split the data strips between them, combining their partial
 * sums in LDS (threads = 64*split; plain code and extended Q parity alike).
 * Only some (vec, unroll) pairs and split factors are built for each prime.
 * The library keeps one process-wide table keyed by (p, op, row-size bucket),
 * bucket = floor(log2(row_bytes)); op 0 = encode, 1 = recovery, 2 and 3 the
 * same for stripes with the extended Q parity (k > p).  Entries
 * change only speed, never results.
 * ------------------------------------------------------------------------ */

/* Bit mask of the vector widths built for prime p (bit v set for vec = v);
 * 0 when p is not built. */
int raid6c_vec_mask(int p);

/* Bit mask of the unroll factors built for (p, vec) (bit u for unroll = u);
 * 0 when the pair is not built. */
int raid6c_unroll_mask(int p, int vec);

/* Bit mask of the split factors built for (p, vec) (bit s for split = s,
 * s = 2, 4); 0 when none is. */
int raid6c_split_mask(int p, int vec);

/* Record the configuration for (p, op, bucket of row_bytes).  order: 0 =
 * work-groups in dispatch order, 1 = renumbered so that runs of neighbouring
 * column tiles go to one XCD (chiplet with its own L2) together, 2 = the
 * stripes of consecutive work-groups spread over the launch (stripe s is
 * handled in place m*s mod n for a fixed m coprime with the n stripes of the
 * launch), so that the work in flight does not sit at the same offsets of
 * neighbouring stripes.  A launch whose rows do not all start on 128-byte
 * lines (row_bytes, strip addresses and strides not multiples of 128) takes
 * order 1 in place of 0 and loads through the caches; otherwise loads are
 * non-temporal.
 * Errors: RAID6C_E_ARG for an unbuilt p, op not 0..3, (vec, unroll) not built
 * for p, threads not 64/128/256, split not 1 or a built factor with
 * threads = 64*split, or order not 0..2. */
int raid6c_tune_set(int p, int op, size_t row_bytes, int vec, int unroll, int threads, int split, int order);

/* The configuration a call with these arguments would use now.
 * Errors: RAID6C_E_ARG for an unbuilt p, op not 0..3, or NULL outputs. */
int raid6c_tune_get(int p, int op, size_t row_bytes, int* vec, int* unroll, int* threads, int* split,
                    int* order);

/* Forget every recorded configuration (back to the built-in rule). */
void raid6c_tune_clear(void);

/* Autotuner for the strided entry points: run every built (vec, unroll,
 * threads, split) configuration on the caller's stripes -- op 0: raid6c_encode_n,
 * op 1: raid6c_recover_n with `erasures` (device, as there) -- once to warm
 * up and `reps` times, each launch timed with HIP events on `stream`, in
 * every work-group order (0, 1 and 2, the latter two for the configurations
 * within 5% of the best), then record the one with the smallest median
 * launch time for (p, op, row-size bucket) -- op + 2 when k > p -- and
 * return that median in *best_ms (may be NULL).  Every run rewrites the same
 * output bytes.
 * Synchronises.  Errors: as raid6c_encode_n / raid6c_recover_n, plus
 * RAID6C_E_ARG for op not 0/1 or reps outside 1..1000, RAID6C_E_HIP. */
int raid6c_autotune_n(int p, int k, size_t row_bytes, void* base,
                      size_t strip_stride, size_t stripe_stride, size_t nstripes,
                      int op, const int32_t* erasures, int reps, void* stream,
                      float* best_ms);

#ifdef __cplusplus
}
#endif

#endif /* RAID6C_H */
