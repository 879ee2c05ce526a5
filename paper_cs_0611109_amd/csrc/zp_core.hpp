// zp_core.hpp -- device code of Z_p-RAID: one (stripe, column tile) of work.
//
// Ring and code: R_p = F2[x]/(1 + x + ... + x^{p-1}), g = x (the Sylvester
// matrix S_p of Lemma 3.4.1), P = sum_t D_t, Q = sum_t g^t D_t
// (Corollary 3.2.4), recovery by the cases of Lemma 3.1.2 with the
// two-data formulas of Sections 4.3 and 4.6.
//
// Layout: a strip is p-1 rows of W bytes.  Every lane (bit) of a row is an
// independent codeword, so a thread owns a V-dword column slice of every row
// of every strip of its stripe and works on whole rows with XOR.
//
// The Q side is computed in C = F2[x]/(x^p - 1) = F2[x]/((x-1)(1+...+x^{p-1})),
// where multiplication by x is a plain cyclic shift of p rows; a strip enters
// C with an extra zero row p-1.  Reducing an element c of C to R_p subtracts
// c[p-1] times (1 + x + ... + x^{p-1}), i.e. XORs row p-1 into every row.  This
// is the closed form of S_p^k in the proof of Lemma 3.4.1 (a rotation plus a
// broadcast of the wrapped row), applied once at the end instead of per step.
//
//  * Streaming phase: for t = k-1 down to 0, acc_q <- x * acc_q + D_t
//    (Horner's rule of Section 4.2 in C: a register rotation, no reduction),
//    and acc_p <- acc_p + D_t.  Every data row is loaded from HBM once and
//    feeds both sums.
//  * Finishing phase, per case: the data-dependent rotations x^{p-x}, x^x and
//    the solve of (1 + x^z) D = T are index permutations of whole rows whose
//    shift is uniform over the stripe; they go through LDS (each thread only
//    touches its own column there, so no barrier is needed).
//
// Solving (1 + x^z) D = T in R_p (z != 0 mod p) without an inverse: lift T to
// C and look for the lift D~ of D with D~[p-1] = 0.  In C the multiples of
// 1 + ... + x^{p-1} are 0 and the all-ones element, so (1 + x^z) D~ = T~ + e*1
// where e is the XOR of all p rows of T~ (both sides have even weight and p is
// odd).  Row u of (1 + x^z) D~ is D~[u] + D~[u-z], hence
//     D~[u] = T~[u] + e + D~[u - z],
// a chain that starts from D~[p-1] = 0 and, because gcd(z, p) = 1, visits the
// rows u = p-1+z, p-1+2z, ... (mod p) once each.  p-1 steps of two XORs
// replace the (p+1)/2-term Horner inverse of Section 4.6.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "raid6c_internal.h"

namespace raid6c {

template <int V> struct vec_t;
template <> struct vec_t<1> { typedef uint32_t type; };
template <> struct vec_t<2> { typedef uint32_t type __attribute__((ext_vector_type(2))); };
template <> struct vec_t<4> { typedef uint32_t type __attribute__((ext_vector_type(4))); };

// Buffer-resource word 3 for raw (untyped, stride 0) buffers on gfx9-class GPUs.
constexpr int kRawBufferWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const uint8_t* base, uint32_t nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(base), (short)0, (int)nbytes,
                                           kRawBufferWord3);
}

// Vector buffer load / store: byte address = base + voff + soff.  The buffer's
// size (one strip) bounds voff in hardware: an access past it reads 0 / is
// dropped instead of touching other memory.
template <int V> struct bufio;
template <> struct bufio<1> {
  typedef uint32_t T;
  static __device__ __forceinline__ T load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
  }
  static __device__ __forceinline__ void store(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(v, r, voff, soff, 0);
  }
};
template <> struct bufio<2> {
  typedef vec_t<2>::type T;
  static __device__ __forceinline__ T load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
  }
  static __device__ __forceinline__ void store(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 0);
  }
};
template <> struct bufio<4> {
  typedef vec_t<4>::type T;
  static __device__ __forceinline__ T load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
  }
  static __device__ __forceinline__ void store(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b128(v, r, voff, soff, 0);
  }
};

// Addresses of one stripe's strips for one thread's column.
struct Cols {
  const ZpArgs* a;
  uint64_t stripe_off;   // stripe * stripe_stride
  uint32_t col;          // byte offset of this thread's slice within a row
  uint32_t strip_bytes;  // (p-1) * row_bytes

  __device__ __forceinline__ __amdgpu_buffer_rsrc_t strip(int j) const {
    return make_rsrc(a->strip[j] + stripe_off, strip_bytes);
  }
};

template <typename VT>
__device__ __forceinline__ VT ld(__amdgpu_buffer_rsrc_t s, int r, uint64_t W, uint32_t col) {
  return bufio<sizeof(VT) / 4>::load(s, col, (uint32_t)r * (uint32_t)W);
}

template <typename VT>
__device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t s, int r, uint64_t W, uint32_t col, VT v) {
  bufio<sizeof(VT) / 4>::store(v, s, col, (uint32_t)r * (uint32_t)W);
}

// Streaming phase over the data strips, skipping strips x and y (-1 = none).
// HP: accumulate acc_p; HQ: accumulate acc_q (Horner in C).
template <int P, int V, bool HP, bool HQ>
__device__ __forceinline__ void stream_data(const Cols& c, int k, int x, int y,
                                            typename vec_t<V>::type (&ap)[P - 1],
                                            typename vec_t<V>::type (&aq)[P]) {
  typedef typename vec_t<V>::type VT;
  constexpr int R = P - 1;
  const uint64_t W = c.a->row_bytes;
  for (int t = k - 1; t >= 0; --t) {
    if (HQ) {
      // acc_q <- x * acc_q in C: cyclic shift of the p rows.
      VT top = aq[P - 1];
#pragma unroll
      for (int u = P - 1; u > 0; --u) aq[u] = aq[u - 1];
      aq[0] = top;
    }
    if (t == x || t == y) continue;
    const __amdgpu_buffer_rsrc_t b = c.strip(t);
    VT v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = ld<VT>(b, r, W, c.col);
    // Keep all p-1 row loads of the strip in flight before the first use.
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (HP) ap[r] ^= v[r];
      if (HQ) aq[r] ^= v[r];
    }
  }
}

template <int P, int V>
__device__ __forceinline__ void load_into(const Cols& c, int j, typename vec_t<V>::type (&acc)[P - 1]) {
  typedef typename vec_t<V>::type VT;
  const __amdgpu_buffer_rsrc_t b = c.strip(j);
  const uint64_t W = c.a->row_bytes;
#pragma unroll
  for (int r = 0; r < P - 1; ++r) acc[r] = ld<VT>(b, r, W, c.col);
}

template <int P, int V>
__device__ __forceinline__ void xor_from(const Cols& c, int j, typename vec_t<V>::type (&acc)[P]) {
  typedef typename vec_t<V>::type VT;
  const __amdgpu_buffer_rsrc_t b = c.strip(j);
  const uint64_t W = c.a->row_bytes;
#pragma unroll
  for (int r = 0; r < P - 1; ++r) acc[r] ^= ld<VT>(b, r, W, c.col);
}

template <int P, int V>
__device__ __forceinline__ void store_strip(const Cols& c, int j, const typename vec_t<V>::type (&v)[P - 1]) {
  typedef typename vec_t<V>::type VT;
  const __amdgpu_buffer_rsrc_t b = c.strip(j);
  const uint64_t W = c.a->row_bytes;
#pragma unroll
  for (int r = 0; r < P - 1; ++r) st<VT>(b, r, W, c.col, v[r]);
}

// Q = reduction of acc_q from C to R_p: row r plus row p-1.
template <int P, int V>
__device__ __forceinline__ void store_reduced(const Cols& c, int j, const typename vec_t<V>::type (&aq)[P]) {
  typedef typename vec_t<V>::type VT;
  const __amdgpu_buffer_rsrc_t b = c.strip(j);
  const uint64_t W = c.a->row_bytes;
  const VT top = aq[P - 1];
#pragma unroll
  for (int r = 0; r < P - 1; ++r) st<VT>(b, r, W, c.col, aq[r] ^ top);
}

// Full encode of one tile: P and Q (either may be skipped).
template <int P, int V>
__device__ __forceinline__ void tile_encode(const Cols& c, int k, bool wp, bool wq) {
  typedef typename vec_t<V>::type VT;
  VT ap[P - 1], aq[P];
#pragma unroll
  for (int r = 0; r < P - 1; ++r) ap[r] = (VT)(0u);
#pragma unroll
  for (int u = 0; u < P; ++u) aq[u] = (VT)(0u);
  if (wp && wq) {
    stream_data<P, V, true, true>(c, k, -1, -1, ap, aq);
  } else if (wp) {
    stream_data<P, V, true, false>(c, k, -1, -1, ap, aq);
  } else {
    stream_data<P, V, false, true>(c, k, -1, -1, ap, aq);
  }
  if (wp) store_strip<P, V>(c, k, ap);
  if (wq) store_reduced<P, V>(c, k + 1, aq);
}

// Recovery of one tile.  `lds` points at this thread's column of a region of
// P rows with a row stride of `ls` vectors; only this thread touches it.
template <int P, int V>
__device__ __forceinline__ void tile_recover(const Cols& c, int k, const Case& cs,
                                             typename vec_t<V>::type* lds, int ls) {
  typedef typename vec_t<V>::type VT;
  constexpr int R = P - 1;
  const int iP = k, iQ = k + 1;

  switch (cs.op) {
    case OP_PQ:
      tile_encode<P, V>(c, k, true, true);
      return;
    case OP_P:
      tile_encode<P, V>(c, k, true, false);
      return;
    case OP_Q:
      tile_encode<P, V>(c, k, false, true);
      return;
    default:
      break;
  }

  VT ap[R], aq[P];
#pragma unroll
  for (int u = 0; u < P; ++u) aq[u] = (VT)(0u);

  if (cs.op == OP_D) {
    // D_x = P + sum_{t != x} D_t.
    load_into<P, V>(c, iP, ap);
    stream_data<P, V, true, false>(c, k, cs.x, -1, ap, aq);
    store_strip<P, V>(c, cs.x, ap);
    return;
  }

  if (cs.op == OP_DQ) {
    // D_x = P + sum_{t != x} D_t;  Q = sum_{t != x} x^t D_t + x^x D_x.
    const int x = cs.x;
    load_into<P, V>(c, iP, ap);
    stream_data<P, V, true, true>(c, k, x, -1, ap, aq);
#pragma unroll
    for (int r = 0; r < R; ++r) lds[r * ls] = ap[r];
    lds[R * ls] = (VT)(0u);
    // (x^x D~)[u] = D~[(u - x) mod p]
#pragma unroll
    for (int u = 0; u < P; ++u) {
      int w = u - x;
      if (w < 0) w += P;
      aq[u] ^= lds[w * ls];
    }
    store_strip<P, V>(c, x, ap);
    store_reduced<P, V>(c, iQ, aq);
    return;
  }

  if (cs.op == OP_DP) {
    // D_x = x^{p-x} (Q + sum_{t != x} x^t D_t);  P = sum_{t != x} D_t + D_x.
    const int x = cs.x;
#pragma unroll
    for (int r = 0; r < R; ++r) ap[r] = (VT)(0u);
    stream_data<P, V, true, true>(c, k, x, -1, ap, aq);
    xor_from<P, V>(c, iQ, aq);
#pragma unroll
    for (int u = 0; u < P; ++u) lds[u * ls] = aq[u];
    // (x^{p-x} a)[u] = a[(u + x) mod p]
    VT d[P];
#pragma unroll
    for (int u = 0; u < P; ++u) {
      int w = u + x;
      if (w >= P) w -= P;
      d[u] = lds[w * ls];
    }
    VT out[R];
#pragma unroll
    for (int r = 0; r < R; ++r) out[r] = d[r] ^ d[R];
    store_strip<P, V>(c, x, out);
#pragma unroll
    for (int r = 0; r < R; ++r) out[r] ^= ap[r];
    store_strip<P, V>(c, iP, out);
    return;
  }

  // OP_DD: data x < y, z = y - x.
  //   dP = P + sum_{t != x,y} D_t,  dQ~ = Q + sum_{t != x,y} x^t D_t (in C),
  //   T~ = dP~ + x^{p-x} dQ~,  (1 + x^z) D_y = T,  D_x = D_y + dP.
  const int x = cs.x;
  const int z = cs.y - cs.x;
  load_into<P, V>(c, iP, ap);
  stream_data<P, V, true, true>(c, k, cs.x, cs.y, ap, aq);
  xor_from<P, V>(c, iQ, aq);

  // e = XOR of all rows of T~ = XOR of all rows of dP~ and of dQ~ (a rotation
  // keeps the set of rows).
  VT e = (VT)(0u);
#pragma unroll
  for (int r = 0; r < R; ++r) e ^= ap[r];
#pragma unroll
  for (int u = 0; u < P; ++u) e ^= aq[u];

  // Chain rows u_s = (p-1 + s z) mod p, s = 1..p-1.
  // T~[u] = dP~[u] + dQ~[(u + x) mod p].
#pragma unroll
  for (int u = 0; u < P; ++u) lds[u * ls] = aq[u];
  VT tch[R];
  {
    int u = R;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      u += z;
      if (u >= P) u -= P;
      int w = u + x;
      if (w >= P) w -= P;
      tch[s] = lds[w * ls];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) lds[r * ls] = ap[r];
  {
    int u = R;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      u += z;
      if (u >= P) u -= P;
      tch[s] ^= lds[u * ls];   // u != p-1 on the chain
    }
  }
  // D~[u_s] = T~[u_s] + e + D~[u_{s-1}],  D~[p-1] = 0.
  {
    VT d = (VT)(0u);
#pragma unroll
    for (int s = 0; s < R; ++s) {
      d = tch[s] ^ e ^ d;
      tch[s] = d;
    }
  }
  {
    int u = R;
#pragma unroll
    for (int s = 0; s < R; ++s) {
      u += z;
      if (u >= P) u -= P;
      lds[u * ls] = tch[s];
    }
  }
  VT dy[R];
#pragma unroll
  for (int r = 0; r < R; ++r) dy[r] = lds[r * ls];
  store_strip<P, V>(c, cs.y, dy);
#pragma unroll
  for (int r = 0; r < R; ++r) dy[r] ^= ap[r];
  store_strip<P, V>(c, cs.x, dy);
}

}  // namespace raid6c
