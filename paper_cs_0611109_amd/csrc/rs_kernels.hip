// rs_kernels.hip -- the conventional Reed-Solomon RAID-6 over GF(256):
// P+Q encode and recovery of any one or two erased disks.
//
// Section 4.1: GF(256) = GF(2)[x]/(x^8+x^4+x^3+x^2+1) (0x11D), g = {02},
// P = sum_t D_t, Q = sum_t g^t D_t bytewise.  Q by Horner's rule
// (Section 4.2): Q <- g Q + D_t for t = k-1 .. 0.  Multiplication by {02}
// shifts each byte left and XORs 0x1D into the bytes whose top bit was set;
// here it is done on four bytes per 32-bit word at once.
//
// Recovery follows the cases of the proof of Lemma 3.1.2 with the cone
// {g^t}: with P_x, Q_x the syndromes of the surviving data disks,
//   data x + P:  D_x = g^{-x} (Q + Q_x), then P = P_x + D_x;
//   data x + Q:  D_x = P + P_x, then Q = Q_x + g^x D_x;
//   data x < y:  D_y = A (P + P_xy) + B (Q + Q_xy), D_x = D_y + P + P_xy with
//                A = (1 + g^{y-x})^{-1}, B = (g^x + g^y)^{-1} (Sections 4.3, 4.4).
// The constants are uniform over a stripe and come from exp/log tables of
// the field; the byte-vector products c*v are done lane-parallel by shift
// and XOR over the bits of c (a scalar loop, since c is uniform), instead of
// the 64 KiB product table of the Linux code.
//
// Grid: one work-group per (stripe, tile); each thread owns V dwords at the
// same offset of every strip of its stripe.  The loads of U strips are all
// issued before the first is used.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "raid6c_internal.h"
#include "zp_core.hpp"

namespace raid6c {

namespace {

// exp[i] = g^i (i = 0..254, exp[255] = exp[0]) and log[g^i] = i, built at
// compile time by repeated multiplication by {02}.
struct GfTables {
  uint8_t exp[256];
  uint8_t log[256];
};

constexpr GfTables make_gf_tables() {
  GfTables t{};
  uint32_t v = 1;
  for (int i = 0; i < 255; ++i) {
    t.exp[i] = (uint8_t)v;
    t.log[v] = (uint8_t)i;
    v <<= 1;
    if (v & 0x100u) v ^= 0x11Du;
  }
  t.exp[255] = t.exp[0];
  return t;
}

__constant__ GfTables kGf = make_gf_tables();

__device__ __forceinline__ uint32_t gf_exp(int e) { return kGf.exp[e % 255]; }
// a^{-1} for a != 0: g^{255 - log a}.
__device__ __forceinline__ uint32_t gf_inv(uint32_t a) { return kGf.exp[(255 - kGf.log[a]) % 255]; }

template <typename VT>
__device__ __forceinline__ VT mul02(VT q) {
  const VT hi = (q >> 7) & (VT)(0x01010101u);
  return ((q & (VT)(0x7f7f7f7fu)) << 1) ^ (hi * (VT)(0x1du));
}

// c * v for a wave-uniform constant c: sum of {02}^i v over the set bits i.
template <typename VT>
__device__ __forceinline__ VT mulc(VT v, uint32_t c) {
  VT acc = (VT)(0u);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    if ((c >> i) & 1u) acc ^= v;
    if ((c >> (i + 1)) == 0u) break;
    v = mul02(v);
  }
  return acc;
}

template <int V, int U>
__global__ void __launch_bounds__(256) rs_kernel(const RsArgs a) {
  typedef typename vec_t<V>::type VT;
  const uint32_t stripe = blockIdx.x / a.tiles;
  const uint32_t tile = blockIdx.x - stripe * a.tiles;
  Case cs{OP_PQ, -1, -1};
  if (a.erasures != nullptr) {
    const int e0 = __builtin_amdgcn_readfirstlane(a.erasures[2 * (uint64_t)stripe]);
    const int e1 = __builtin_amdgcn_readfirstlane(a.erasures[2 * (uint64_t)stripe + 1]);
    cs = classify(a.k, e0, e1);
    if (cs.op == OP_BAD) {
      if (tile == 0 && threadIdx.x == 0 && a.bad_count != nullptr) atomicAdd(a.bad_count, 1);
      return;
    }
  }
  const int op = __builtin_amdgcn_readfirstlane(cs.op);
  const int x = __builtin_amdgcn_readfirstlane(cs.x);
  const int y = __builtin_amdgcn_readfirstlane(cs.y);
  const uint32_t off = (tile * blockDim.x + threadIdx.x) * (V * 4);
  if (off >= a.strip_bytes) return;
  uint8_t* const s = a.base + (uint64_t)stripe * a.stripe_stride;
  const uint32_t nb = (uint32_t)a.strip_bytes;
  auto strip = [&](int j) { return make_rsrc(s + (uint64_t)j * a.strip_stride, nb); };
  const int k = a.k;

  // Syndromes over the data disks other than x and y (P_xy, Q_xy).
  VT p = (VT)(0u), q = (VT)(0u);
  int t = k - 1;
#pragma unroll 1
  for (; t >= U - 1; t -= U) {
    __builtin_amdgcn_sched_barrier(0);
    VT v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int tt = t - u;
      v[u] = (tt == x || tt == y) ? (VT)(0u) : bufio<V>::load(strip(tt), off, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      p ^= v[u];
      q = mul02(q) ^ v[u];
    }
  }
#pragma unroll 1
  for (; t >= 0; --t) {
    const VT d = (t == x || t == y) ? (VT)(0u) : bufio<V>::load(strip(t), off, 0);
    p ^= d;
    q = mul02(q) ^ d;
  }

  const int iP = k, iQ = k + 1;
  switch (op) {
    case OP_PQ:
      bufio<V>::store(p, strip(iP), off, 0);
      bufio<V>::store(q, strip(iQ), off, 0);
      return;
    case OP_P:
      bufio<V>::store(p, strip(iP), off, 0);
      return;
    case OP_Q:
      bufio<V>::store(q, strip(iQ), off, 0);
      return;
    case OP_D:
      bufio<V>::store(p ^ bufio<V>::load(strip(iP), off, 0), strip(x), off, 0);
      return;
    case OP_DQ: {
      const VT d = p ^ bufio<V>::load(strip(iP), off, 0);
      bufio<V>::store(d, strip(x), off, 0);
      bufio<V>::store(q ^ mulc(d, gf_exp(x)), strip(iQ), off, 0);
      return;
    }
    case OP_DP: {
      const VT d = mulc(q ^ bufio<V>::load(strip(iQ), off, 0), gf_exp(255 - x));
      bufio<V>::store(d, strip(x), off, 0);
      bufio<V>::store(p ^ d, strip(iP), off, 0);
      return;
    }
    default: {  // OP_DD
      const VT dp = p ^ bufio<V>::load(strip(iP), off, 0);
      const VT dq = q ^ bufio<V>::load(strip(iQ), off, 0);
      const uint32_t A = gf_inv(1u ^ gf_exp(y - x));
      const uint32_t B = gf_inv(gf_exp(x) ^ gf_exp(y));
      const VT dy = mulc(dp, A) ^ mulc(dq, B);
      bufio<V>::store(dy, strip(y), off, 0);
      bufio<V>::store(dy ^ dp, strip(x), off, 0);
      return;
    }
  }
}

template <int V>
hipError_t launch_v(const RsArgs& a, int unroll, int threads, uint32_t grid, hipStream_t stream) {
  const dim3 g(grid), b(threads);
  switch (unroll) {
    case 1: hipLaunchKernelGGL((rs_kernel<V, 1>), g, b, 0, stream, a); break;
    case 4: hipLaunchKernelGGL((rs_kernel<V, 4>), g, b, 0, stream, a); break;
    case 8: hipLaunchKernelGGL((rs_kernel<V, 8>), g, b, 0, stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t rs_launch(const RsArgs& a, int vec, int unroll, int threads, uint32_t grid, hipStream_t stream) {
  switch (vec) {
    case 1: return launch_v<1>(a, unroll, threads, grid, stream);
    case 2: return launch_v<2>(a, unroll, threads, grid, stream);
    case 4: return launch_v<4>(a, unroll, threads, grid, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace raid6c
