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
// thread's LDS column, one dword column at a time.  Rows that do not all
// start on 128-byte lines (SHARED) load with the ordinary cache policy and
// take the XCD-chunked work-group order, as the encode and recovery kernels
// do: a line at the edge of two tiles is then fetched once into one L2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "raid6c_internal.h"
#include "zp_core.hpp"

namespace raid6c {

namespace {

template <int P, int V, bool SHARED>
__global__ void __launch_bounds__(256) update_kernel(const UpdArgs a) {
  typedef typename vec_t<V>::type VT;
  typedef comp<V> CP;
  constexpr int R = P - 1;
  constexpr int LP = SHARED ? kLoadPolicyShared : RAID6C_LOAD_POLICY;
  extern __shared__ __align__(16) uint32_t smem[];
  const uint32_t b = SHARED ? xcd_chunk(blockIdx.x, gridDim.x) : blockIdx.x;
  const uint32_t stripe = b / a.tiles;
  const uint32_t tile = b - stripe * a.tiles;
  const uint32_t col = (tile * blockDim.x + threadIdx.x) * (V * 4);
  const uint64_t W = a.row_bytes;
  const uint32_t nb = (uint32_t)(R * W);
  uint8_t *sb = nullptr, *pp, *pq;
  if (a.base != nullptr) {
    sb = a.base + (uint64_t)stripe * a.stripe_stride;
    pp = sb + (uint64_t)a.k * a.strip_stride;
    pq = sb + (uint64_t)(a.k + 1) * a.strip_stride;
  } else {
    pp = a.pp;
    pq = a.pq;
  }
  const __amdgpu_buffer_rsrc_t bp = make_rsrc(pp, nb), bq = make_rsrc(pq, nb);
  const __amdgpu_buffer_rsrc_t bn = make_rsrc(a.src + (uint64_t)stripe * a.src_stride, nb);
  const bool live = col < a.row_bytes;

  // The new strip, P and Q do not depend on which strip is replaced: their
  // loads go out first, while the target index is still on its way.
  VT n[R], pr[R], q[R];
  if (live) {
#pragma unroll
    for (int r = 0; r < R; ++r) n[r] = ld<VT, LP>(bn, r, W, col);
#pragma unroll
    for (int r = 0; r < R; ++r) pr[r] = ld<VT, LP>(bp, r, W, col);
#pragma unroll
    for (int r = 0; r < R; ++r) q[r] = ld<VT, LP>(bq, r, W, col);
  }
  int t = a.t;
  if (a.targets != nullptr) t = a.targets[stripe];
  t = __builtin_amdgcn_readfirstlane(t);
  if (t < 0 || t >= a.k) {
    if (tile == 0 && threadIdx.x == 0 && a.bad_count != nullptr) atomicAdd(a.bad_count, 1);
    return;
  }
  if (!live) return;
  uint8_t* pd = sb != nullptr ? sb + (uint64_t)t * a.strip_stride : a.pd;
  const __amdgpu_buffer_rsrc_t bd = make_rsrc(pd, nb);

  VT d[R];
#pragma unroll
  for (int r = 0; r < R; ++r) d[r] = ld<VT, LP>(bd, r, W, col);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    d[r] ^= n[r];
    st<VT>(bd, r, W, col, n[r]);
    st<VT>(bp, r, W, col, pr[r] ^ d[r]);
  }
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

template <int P, bool SHARED>
hipError_t launch_ps(const UpdArgs& a, int vec, int threads, uint32_t grid, hipStream_t stream) {
  const size_t lds = (size_t)P * threads * 4;
  if (vec == 1) {
    hipLaunchKernelGGL((update_kernel<P, 1, SHARED>), dim3(grid), dim3(threads), lds, stream, a);
  } else if (vec == 2 && P <= 31) {
    hipLaunchKernelGGL((update_kernel<P, (P <= 31 ? 2 : 1), SHARED>), dim3(grid), dim3(threads), lds, stream, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int P>
hipError_t launch_p(const UpdArgs& a, int vec, int threads, uint32_t grid, bool shared_lines, hipStream_t stream) {
  return shared_lines ? launch_ps<P, true>(a, vec, threads, grid, stream)
                      : launch_ps<P, false>(a, vec, threads, grid, stream);
}

}  // namespace

hipError_t update_launch(const UpdArgs& a, int p, int vec, int threads, uint32_t grid, bool shared_lines,
                         hipStream_t stream) {
  switch (p) {
#define RAID6C_UPD(q) \
  case q:             \
    return launch_p<q>(a, vec, threads, grid, shared_lines, stream);
    RAID6C_UPD(3) RAID6C_UPD(5) RAID6C_UPD(7) RAID6C_UPD(11) RAID6C_UPD(13) RAID6C_UPD(17) RAID6C_UPD(19)
    RAID6C_UPD(23) RAID6C_UPD(29) RAID6C_UPD(31) RAID6C_UPD(37) RAID6C_UPD(41) RAID6C_UPD(43) RAID6C_UPD(47)
    RAID6C_UPD(53) RAID6C_UPD(59) RAID6C_UPD(61)
#undef RAID6C_UPD
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace raid6c
