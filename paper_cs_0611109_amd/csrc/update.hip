// update.hip -- small writes: one data strip of a stripe is replaced and the
// parities follow from the change alone.  The parity equations of
// Corollary 3.2.4 are linear, so with dD = D_t + D_t'
//   P' = P + dD,   Q' = Q + g_t dD,
// g_t = x^t, or 1 + x^{t-p+1} for a strip t >= p of the extended Q parity
// (Section 3.3); multiplying by a power of x is the rotation-and-broadcast
// of Lemma 3.4.1 that the end of Section 3.4 prices for Q-parity updates.
// A stripe reads the old strip, the new one, P and Q and writes the strip,
// P and Q: seven strips, whatever k is.
//
// Grid: one work-group per (stripe, column tile); each thread owns V dwords
// of every row.  The data-dependent rotation of dD goes through the
// thread's LDS column, one dword column at a time.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "raid6c_internal.h"
#include "zp_core.hpp"

namespace raid6c {

namespace {

template <int P, int V>
__global__ void __launch_bounds__(256) update_kernel(const UpdArgs a) {
  typedef typename vec_t<V>::type VT;
  typedef comp<V> CP;
  constexpr int R = P - 1;
  extern __shared__ __align__(16) uint32_t smem[];
  const uint32_t stripe = blockIdx.x / a.tiles;
  const uint32_t tile = blockIdx.x - stripe * a.tiles;
  int t = a.t;
  if (a.targets != nullptr) t = a.targets[stripe];
  t = __builtin_amdgcn_readfirstlane(t);
  if (t < 0 || t >= a.k) {
    if (tile == 0 && threadIdx.x == 0 && a.bad_count != nullptr) atomicAdd(a.bad_count, 1);
    return;
  }
  const uint32_t col = (tile * blockDim.x + threadIdx.x) * (V * 4);
  if (col >= a.row_bytes) return;
  const uint64_t W = a.row_bytes;
  const uint32_t nb = (uint32_t)(R * W);
  uint8_t *pd, *pp, *pq;
  if (a.base != nullptr) {
    uint8_t* sb = a.base + (uint64_t)stripe * a.stripe_stride;
    pd = sb + (uint64_t)t * a.strip_stride;
    pp = sb + (uint64_t)a.k * a.strip_stride;
    pq = sb + (uint64_t)(a.k + 1) * a.strip_stride;
  } else {
    pd = a.pd;
    pp = a.pp;
    pq = a.pq;
  }
  const __amdgpu_buffer_rsrc_t bd = make_rsrc(pd, nb), bp = make_rsrc(pp, nb), bq = make_rsrc(pq, nb);
  const __amdgpu_buffer_rsrc_t bn = make_rsrc(a.src + (uint64_t)stripe * a.src_stride, nb);

  VT d[R], n[R], pr[R];
#pragma unroll
  for (int r = 0; r < R; ++r) d[r] = ld<VT>(bd, r, W, col);
#pragma unroll
  for (int r = 0; r < R; ++r) n[r] = ld<VT>(bn, r, W, col);
#pragma unroll
  for (int r = 0; r < R; ++r) pr[r] = ld<VT>(bp, r, W, col);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    d[r] ^= n[r];
    st<VT>(bd, r, W, col, n[r]);
    st<VT>(bp, r, W, col, pr[r] ^ d[r]);
  }
  VT q[R];
#pragma unroll
  for (int r = 0; r < R; ++r) q[r] = ld<VT>(bq, r, W, col);
  // g_t dD: rotation by s of the lift of dD in C, reduced (row r plus the
  // row that lands on p-1); plus dD itself for an extended strip.
  const bool ext = t >= P;
  const int s = ext ? t - P + 1 : t;
  uint32_t* lds = smem + threadIdx.x;
  const int ls = (int)blockDim.x;
#pragma unroll
  for (int cc = 0; cc < V; ++cc) {
#pragma unroll
    for (int r = 0; r < R; ++r) lds[r * ls] = CP::get(d[r], cc);
    lds[R * ls] = 0u;
    const uint32_t top = lds[(R - s) * ls];   // (x^s dD~)[p-1] = dD~[p-1-s]
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int w = r - s;
      if (w < 0) w += P;
      uint32_t v = lds[w * ls] ^ top;
      if (ext) v ^= CP::get(d[r], cc);
      CP::set(q[r], cc, CP::get(q[r], cc) ^ v);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) st<VT>(bq, r, W, col, q[r]);
}

template <int P>
hipError_t launch_p(const UpdArgs& a, int vec, int threads, uint32_t grid, hipStream_t stream) {
  const size_t lds = (size_t)P * threads * 4;
  if (vec == 1) {
    hipLaunchKernelGGL((update_kernel<P, 1>), dim3(grid), dim3(threads), lds, stream, a);
  } else if (vec == 2 && P <= 31) {
    hipLaunchKernelGGL((update_kernel<P, (P <= 31 ? 2 : 1)>), dim3(grid), dim3(threads), lds, stream, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t update_launch(const UpdArgs& a, int p, int vec, int threads, uint32_t grid, hipStream_t stream) {
  switch (p) {
#define RAID6C_UPD(q) \
  case q:             \
    return launch_p<q>(a, vec, threads, grid, stream);
    RAID6C_UPD(3) RAID6C_UPD(5) RAID6C_UPD(7) RAID6C_UPD(11) RAID6C_UPD(13) RAID6C_UPD(17) RAID6C_UPD(19)
    RAID6C_UPD(23) RAID6C_UPD(29) RAID6C_UPD(31) RAID6C_UPD(37) RAID6C_UPD(41) RAID6C_UPD(43) RAID6C_UPD(47)
    RAID6C_UPD(53) RAID6C_UPD(59) RAID6C_UPD(61)
#undef RAID6C_UPD
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace raid6c
