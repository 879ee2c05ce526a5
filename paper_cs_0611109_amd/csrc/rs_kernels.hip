// rs_kernels.hip -- the conventional Reed-Solomon P+Q encode over GF(256).
//
// Section 4.1: GF(256) = GF(2)[x]/(x^8+x^4+x^3+x^2+1) (0x11D), g = {02},
// P = sum_t D_t, Q = sum_t g^t D_t bytewise.  Q by Horner's rule
// (Section 4.2): Q <- g Q + D_t for t = k-1 .. 0.  Multiplication by {02}
// shifts each byte left and XORs 0x1D into the bytes whose top bit was set;
// here it is done on four bytes per 32-bit word at once.
//
// Grid: one work-group per (stripe, tile); each thread owns V dwords at the
// same offset of every strip of its stripe.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "raid6c_internal.h"
#include "zp_core.hpp"

namespace raid6c {

namespace {

template <typename VT>
__device__ __forceinline__ VT mul02(VT q) {
  const VT hi = (q >> 7) & (VT)(0x01010101u);
  return ((q & (VT)(0x7f7f7f7fu)) << 1) ^ (hi * (VT)(0x1du));
}

template <int V>
__global__ void __launch_bounds__(256) rs_encode_kernel(const RsArgs a) {
  typedef typename vec_t<V>::type VT;
  const uint32_t stripe = blockIdx.x / a.tiles;
  const uint32_t tile = blockIdx.x - stripe * a.tiles;
  const uint32_t off = (tile * blockDim.x + threadIdx.x) * (V * 4);
  if (off >= a.strip_bytes) return;
  uint8_t* s = a.base + (uint64_t)stripe * a.stripe_stride;
  VT p = (VT)(0u), q = (VT)(0u);
#pragma unroll 4
  for (int t = a.k - 1; t >= 0; --t) {
    const VT d = *reinterpret_cast<const VT*>(s + (uint64_t)t * a.strip_stride + off);
    p ^= d;
    q = mul02(q) ^ d;
  }
  *reinterpret_cast<VT*>(s + (uint64_t)a.k * a.strip_stride + off) = p;
  *reinterpret_cast<VT*>(s + (uint64_t)(a.k + 1) * a.strip_stride + off) = q;
}

}  // namespace

hipError_t rs_launch(const RsArgs& a, int vec, int threads, uint32_t grid, hipStream_t stream) {
  const dim3 g(grid), b(threads);
  switch (vec) {
    case 1:
      hipLaunchKernelGGL(rs_encode_kernel<1>, g, b, 0, stream, a);
      break;
    case 2:
      hipLaunchKernelGGL(rs_encode_kernel<2>, g, b, 0, stream, a);
      break;
    case 4:
      hipLaunchKernelGGL(rs_encode_kernel<4>, g, b, 0, stream, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace raid6c
