// zp_multi.h -- the job-list kernel for the small groups of every prime up
// to kMultiMaxPrime in one grid (zp_multi.hip).
#pragma once

namespace raid6c {

constexpr int kMultiMaxPrime = 31;

// __global__ void(GroupArgs): one item per work-group of 256 threads; items
// are tiles of 64 lanes x zp_multi_vec(p) dwords of a plain-code job with
// p <= kMultiMaxPrime; zp_multi_lds(p) bytes of dynamic LDS cover every job
// of that prime or a smaller one.
const void* zp_multi_kernel();
int zp_multi_vec(int p);
int zp_multi_lds(int p);

}  // namespace raid6c
