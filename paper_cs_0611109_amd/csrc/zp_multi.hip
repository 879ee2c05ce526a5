// zp_multi.hip -- one job-list kernel for the small groups of every prime up
// to 31, dispatched on each item's prime.
//
// The request server launches, per phase of a batch, one grid per prime
// present.  Each such grid is too small to fill the GPU, and grids on one
// stream run one after another, so a phase lasts as long as its grids' walks
// added up.  Here the plain-code groups of all primes up to 31 that would
// take the latency kernel go into one grid instead; they run side by side.
//
// Every item is one column tile of one job, taken by a work-group of four
// waves that split the job's strips (tile_split, as the per-prime latency
// kernels do), with the per-prime vector width of those kernels: vec 2 up
// to p = 13, vec 1 above.  The four partials of the largest prime fit in
// 64 KiB of LDS up to p = 31; the host gives each launch the LDS of the
// largest prime it holds.  Registers are those of the largest case, which
// is fine for grids that hold far fewer waves than the GPU runs at once.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "raid6c_internal.h"
#include "zp_core.hpp"
#include "zp_multi.h"

namespace raid6c {

namespace {

constexpr int multi_vec(int p) { return p <= 13 ? 2 : 1; }
constexpr int multi_lds(int p) { return 4 * (2 * p - 1) * 64 * multi_vec(p) * 4; }
static_assert(multi_lds(kMultiMaxPrime) <= 65536, "split partials exceed 64 KiB of LDS");

template <int P>
__device__ __forceinline__ void multi_item(const BatchItem& item, const BatchJob& j, uint32_t* part) {
  constexpr int V = multi_vec(P);
  const uint32_t col = item.col + (threadIdx.x & 63) * (V * 4);
  const ColsJob c{j.base, j.strip_stride, j.out0, j.out1, j.src, j.src_stride, j.e0, j.e1,
                  j.row_bytes, col, (uint32_t)((P - 1) * j.row_bytes)};
  const Case cs{j.op, j.x, j.y};
  if (c.lines_aligned())
    tile_split<P, V, 4, 4, false>(c, j.k, cs, item.col, part);
  else
    tile_split<P, V, 4, 4, false>(c.with_policy<kLoadPolicyShared>(), j.k, cs, item.col, part);
}

// One item per work-group of four waves (plain code, p <= kMultiMaxPrime).
__global__ void __launch_bounds__(256) zp_group_multi_kernel(const GroupArgs a) {
  extern __shared__ __align__(16) uint32_t part[];
  const uint32_t i = xcd_chunk(blockIdx.x, gridDim.x);
  if (i >= a.nitems) return;   // uniform over the work-group
  const BatchItem item = a.items[i];
  const BatchJob& j = a.jobs[item.job];
  switch (__builtin_amdgcn_readfirstlane(j.p)) {
#define RAID6C_MULTI_CASE(q)       \
  case q:                          \
    multi_item<q>(item, j, part);  \
    break;
    RAID6C_MULTI_CASE(3)
    RAID6C_MULTI_CASE(5)
    RAID6C_MULTI_CASE(7)
    RAID6C_MULTI_CASE(11)
    RAID6C_MULTI_CASE(13)
    RAID6C_MULTI_CASE(17)
    RAID6C_MULTI_CASE(19)
    RAID6C_MULTI_CASE(23)
    RAID6C_MULTI_CASE(29)
    RAID6C_MULTI_CASE(31)
#undef RAID6C_MULTI_CASE
    default:
      break;
  }
}

}  // namespace

const void* zp_multi_kernel() { return (const void*)zp_group_multi_kernel; }
int zp_multi_vec(int p) { return multi_vec(p); }
int zp_multi_lds(int p) { return multi_lds(p); }

}  // namespace raid6c
