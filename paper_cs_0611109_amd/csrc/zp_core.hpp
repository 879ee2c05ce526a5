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

// Cache-policy operand of the buffer loads and stores.  Every byte is read
// or written exactly once, so both are marked non-temporal (bit 1, "nt" on
// gfx94x/gfx950): streamed through without displacing cache lines.
#ifndef RAID6C_LOAD_POLICY
#define RAID6C_LOAD_POLICY 2
#endif
// Loads of stripes whose rows do not start on 128-byte cache lines: a wave's
// slice of a row then straddles a line that the neighbouring tile's wave
// also reads.  Non-temporal loads let that line go before the second read
// and it is fetched twice (up to 1.4x the bytes at 256-byte slices);
// ordinary loads keep part of those lines for the second reader.
#ifndef RAID6C_SHARED_LOAD_POLICY
#define RAID6C_SHARED_LOAD_POLICY 0
#endif
constexpr int kLoadPolicyShared = RAID6C_SHARED_LOAD_POLICY;
#ifndef RAID6C_STORE_POLICY
#define RAID6C_STORE_POLICY 2
#endif

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
  template <int LP = RAID6C_LOAD_POLICY>
  static __device__ __forceinline__ T load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, LP);
  }
  static __device__ __forceinline__ void store(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(v, r, voff, soff, RAID6C_STORE_POLICY);
  }
};
template <> struct bufio<2> {
  typedef vec_t<2>::type T;
  template <int LP = RAID6C_LOAD_POLICY>
  static __device__ __forceinline__ T load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, LP);
  }
  static __device__ __forceinline__ void store(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, RAID6C_STORE_POLICY);
  }
};
template <> struct bufio<4> {
  typedef vec_t<4>::type T;
  template <int LP = RAID6C_LOAD_POLICY>
  static __device__ __forceinline__ T load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, LP);
  }
  // Stored as two 8-byte halves.  A buffer store of more than 8 bytes whose
  // data registers are rewritten by the very next vector ALU instructions
  // needs a wait state that the compiler does not insert when the store's
  // offset comes from a scalar register; on gfx950 that produced wrong bytes
  // in the last dword of a few lanes.  8-byte stores are not affected.
  static __device__ __forceinline__ void store(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    typedef vec_t<2>::type H;
    // The halves use different scalar offsets so that they are not merged
    // back into one 16-byte store.
    __builtin_amdgcn_raw_buffer_store_b64(H{v.x, v.y}, r, voff, soff, RAID6C_STORE_POLICY);
    __builtin_amdgcn_raw_buffer_store_b64(H{v.z, v.w}, r, voff, soff + 8u, RAID6C_STORE_POLICY);
  }
};

// Work-groups are handed to the 8 XCDs, each with its own L2, round-robin:
// work-group b runs on XCD b mod 8.  xcd_chunk renumbers them so that runs
// of RAID6C_XCD_CHUNK consecutive logical work-groups (neighbouring tiles)
// run on one XCD at about the same time: a cache line at the edge of two
// tiles (rows not on 128-byte lines) is then fetched into one L2, not two.
// Full super-blocks of 8 * chunk work-groups are permuted within
// themselves, so the load stays spread; the tail keeps its numbers.
#ifndef RAID6C_XCD_CHUNK
#define RAID6C_XCD_CHUNK 16
#endif
__device__ __forceinline__ uint32_t xcd_chunk(uint32_t b, uint32_t g) {
#if RAID6C_XCD_CHUNK > 0
  constexpr uint32_t C = RAID6C_XCD_CHUNK, SB = 8u * C;
  if (b >= g / SB * SB) return b;
  const uint32_t x = b % 8u, i = b / 8u;
  return (i / C) * SB + x * C + i % C;
#else
  (void)g;
  return b;
#endif
}

// Where one stripe's strips are, for one thread's column slice.  Both forms
// offer strip(j) (a buffer resource over strip j, the place the stripe's
// strip lives and results are written), src(j) (where data strip j is read
// from: strip(j), or a separate source when the stripe is being written from
// a payload), copy() (true when src differs from strip, so data rows read from
// src are also stored to strip), W() (row bytes) and col (this thread's byte
// offset within a row), and kLoad, the cache policy of their loads.
//  * ColsTableP<LP>: a table of k+2 strip addresses (kernel argument) plus a
//    per-stripe offset; an optional source table for writes.
//  * ColsJobP<LP>: strip j at base + j * strip_stride except that the erased
//    strips e0, e1 may be redirected to out0, out1 (a degraded read rebuilds
//    them into a separate buffer); an optional contiguous source for writes.
template <int LP>
struct ColsTableP {
  static constexpr int kLoad = LP;
  const ZpArgs* a;
  uint64_t stripe_off;   // stripe * stripe_stride
  uint64_t src_off;      // stripe * src_stripe_stride
  uint32_t col;
  uint32_t strip_bytes;  // (p-1) * row_bytes

  __device__ __forceinline__ __amdgpu_buffer_rsrc_t strip(int j) const {
    return make_rsrc(a->strip[j] + stripe_off, strip_bytes);
  }
  __device__ __forceinline__ bool copy() const { return a->src_base != nullptr; }
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t src(int j) const {
    return copy() ? make_rsrc(a->src_base + src_off + (uint64_t)j * a->src_strip_stride, strip_bytes) : strip(j);
  }
  __device__ __forceinline__ uint64_t W() const { return a->row_bytes; }
};
typedef ColsTableP<RAID6C_LOAD_POLICY> ColsTable;

template <int LP>
struct ColsJobP {
  static constexpr int kLoad = LP;
  uint8_t* base;
  uint64_t strip_stride;
  uint8_t* out0;         // where strip e0 is written (base + e0 * strip_stride in place)
  uint8_t* out1;
  const uint8_t* src_base;  // data source of a write, or NULL
  uint64_t src_stride;
  int e0, e1;
  uint32_t row_bytes;
  uint32_t col;
  uint32_t strip_bytes;

  __device__ __forceinline__ __amdgpu_buffer_rsrc_t strip(int j) const {
    // Two one-sided choices: a choice between the two fields out0 / out1
    // can be compiled as one load from a computed field address, which
    // keeps the whole object in private memory.
    uint8_t* p = base + (uint64_t)j * strip_stride;
    p = j == e0 ? out0 : p;
    p = j == e1 ? out1 : p;
    return make_rsrc(p, strip_bytes);
  }
  __device__ __forceinline__ bool copy() const { return src_base != nullptr; }
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t src(int j) const {
    return copy() ? make_rsrc(src_base + (uint64_t)j * src_stride, strip_bytes)
                  : make_rsrc(base + (uint64_t)j * strip_stride, strip_bytes);
  }
  __device__ __forceinline__ uint64_t W() const { return row_bytes; }
  template <int LP2>
  __device__ __forceinline__ ColsJobP<LP2> with_policy() const {
    return ColsJobP<LP2>{base, strip_stride, out0, out1, src_base, src_stride, e0, e1, row_bytes, col, strip_bytes};
  }
  // True when every row of every strip starts on a 128-byte line.
  __device__ __forceinline__ bool lines_aligned() const {
    return (((uintptr_t)base | strip_stride | row_bytes | (uintptr_t)out0 | (uintptr_t)out1 |
             (uintptr_t)src_base | src_stride) & 127u) == 0;
  }
};
typedef ColsJobP<RAID6C_LOAD_POLICY> ColsJob;

// Row r of a strip: the row offset r*W is the same for the whole wave and is
// the scalar offset operand of the buffer instruction.  With
// RAID6C_UNIFORM_ROW_HINT, readfirstlane states that it is uniform: in the
// extended-parity kernels the compiler otherwise keeps such offsets in
// vector registers and wraps every access in a loop over the distinct
// values.  (Elsewhere the hint is not needed, and in the persistent kernel
// it makes compilation very slow.)
#ifndef RAID6C_UNIFORM_ROW_HINT
#define RAID6C_UNIFORM_ROW_HINT 0
#endif
__device__ __forceinline__ uint32_t row_offset(int r, uint64_t W) {
  const uint32_t o = (uint32_t)r * (uint32_t)W;
#if RAID6C_UNIFORM_ROW_HINT
  return __builtin_amdgcn_readfirstlane(o);
#else
  return o;
#endif
}

template <typename VT, int LP = RAID6C_LOAD_POLICY>
__device__ __forceinline__ VT ld(__amdgpu_buffer_rsrc_t s, int r, uint64_t W, uint32_t col) {
  return bufio<sizeof(VT) / 4>::template load<LP>(s, col, row_offset(r, W));
}

template <typename VT>
__device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t s, int r, uint64_t W, uint32_t col, VT v) {
  bufio<sizeof(VT) / 4>::store(v, s, col, row_offset(r, W));
}

// acc_q <- x * acc_q in C: a cyclic shift of the p rows (register renaming).
template <int P, typename VT>
__device__ __forceinline__ void rotate_up(VT (&aq)[P]) {
  const VT top = aq[P - 1];
#pragma unroll
  for (int u = P - 1; u > 0; --u) aq[u] = aq[u - 1];
  aq[0] = top;
}

// Streaming over the data strips hi down to lo, skipping strips x and y
// (-1 = none).  HP: accumulate acc_p; HQ: accumulate acc_q (Horner in C).
// The strips are taken U at a time: the U*(p-1) row loads of a batch are all
// issued before the first of them is used, so each thread keeps U*(p-1)
// loads in flight.
template <int P, int V, int U, bool HP, bool HQ, class C>
__device__ __forceinline__ void stream_range(const C& c, int hi, int lo, int x, int y,
                                             typename vec_t<V>::type (&ap)[P - 1],
                                             typename vec_t<V>::type (&aq)[P]) {
  typedef typename vec_t<V>::type VT;
  constexpr int R = P - 1;
  const uint64_t W = c.W();
  int t = hi;
  // Never unrolled: with constant bounds (the p strips below p of an
  // extended stripe) the compiler would otherwise hoist every load of the
  // range at once.
#pragma unroll 1
  for (; t >= lo + U - 1; t -= U) {
    __builtin_amdgcn_sched_barrier(0);
    VT v[U][R];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int tt = t - u;
      if (tt == x || tt == y) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[u][r] = (VT)(0u);
      } else {
        const __amdgpu_buffer_rsrc_t b = c.src(tt);
#pragma unroll
        for (int r = 0; r < R; ++r) v[u][r] = ld<VT, C::kLoad>(b, r, W, c.col);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    if (c.copy()) {
      // Writing a stripe from a payload: the data rows go to the stripe too.
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int tt = t - u;
        if (tt == x || tt == y) continue;
        const __amdgpu_buffer_rsrc_t d = c.strip(tt);
#pragma unroll
        for (int r = 0; r < R; ++r) st<VT>(d, r, W, c.col, v[u][r]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (HQ) rotate_up<P>(aq);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (HP) ap[r] ^= v[u][r];
        if (HQ) aq[r] ^= v[u][r];
      }
    }
  }
#pragma unroll 1
  for (; t >= lo; --t) {
    if (HQ) rotate_up<P>(aq);
    __builtin_amdgcn_sched_barrier(0);
    if (t == x || t == y) continue;
    const __amdgpu_buffer_rsrc_t b = c.src(t);
    VT v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = ld<VT, C::kLoad>(b, r, W, c.col);
    __builtin_amdgcn_sched_barrier(0);
    if (c.copy()) {
      const __amdgpu_buffer_rsrc_t d = c.strip(t);
#pragma unroll
      for (int r = 0; r < R; ++r) st<VT>(d, r, W, c.col, v[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (HP) ap[r] ^= v[r];
      if (HQ) aq[r] ^= v[r];
    }
  }
}

// The whole streaming phase over data strips k-1 .. 0.
//  * Plain code (EXT false, k <= p): one Horner pass.
//  * Extended Q parity (EXT true, p < k <= 2p-1; Section 3.3, eq. qext):
//    strip t >= p enters Q with 1 + x^{t-p+1}.  A Horner pass over those
//    strips leaves A = sum_{t>=p} x^{t-p} D_t in acc_q while acc_p collects
//    B = sum_{t>=p} D_t; then acc_q <- x A + B, and the pass over the p
//    strips t < p multiplies that by x^p = 1 (in C) while adding
//    sum_{t<p} x^t D_t.  acc_p must start at zero in this case.
template <int P, int V, int U, bool HP, bool HQ, bool EXT, class C>
__device__ __forceinline__ void stream_data(const C& c, int k, int x, int y,
                                            typename vec_t<V>::type (&ap)[P - 1],
                                            typename vec_t<V>::type (&aq)[P]) {
  if constexpr (!EXT) {
    stream_range<P, V, U, HP, HQ>(c, k - 1, 0, x, y, ap, aq);
  } else {
    stream_range<P, V, U, HP || HQ, HQ>(c, k - 1, P, x, y, ap, aq);
    if (HQ) {
      rotate_up<P>(aq);
#pragma unroll
      for (int r = 0; r < P - 1; ++r) aq[r] ^= ap[r];
    }
    stream_range<P, V, U, HP, HQ>(c, P - 1, 0, x, y, ap, aq);
  }
}

template <int P, int V, class C>
__device__ __forceinline__ void load_into(const C& c, int j, typename vec_t<V>::type (&acc)[P - 1]) {
  typedef typename vec_t<V>::type VT;
  const __amdgpu_buffer_rsrc_t b = c.strip(j);
  const uint64_t W = c.W();
#pragma unroll
  for (int r = 0; r < P - 1; ++r) acc[r] = ld<VT, C::kLoad>(b, r, W, c.col);
  __builtin_amdgcn_sched_barrier(0);
}

// acc[r] ^= strip j row r, r < p-1 (acc has p-1 or p entries).
template <int P, int V, int N, class C>
__device__ __forceinline__ void xor_from(const C& c, int j, typename vec_t<V>::type (&acc)[N]) {
  typedef typename vec_t<V>::type VT;
  const __amdgpu_buffer_rsrc_t b = c.strip(j);
  const uint64_t W = c.W();
  VT v[P - 1];
#pragma unroll
  for (int r = 0; r < P - 1; ++r) v[r] = ld<VT, C::kLoad>(b, r, W, c.col);
  // All rows in flight before the first use (as in the streaming phase).
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int r = 0; r < P - 1; ++r) acc[r] ^= v[r];
}

template <int P, int V, class C>
__device__ __forceinline__ void store_strip(const C& c, int j, const typename vec_t<V>::type (&v)[P - 1]) {
  typedef typename vec_t<V>::type VT;
  const __amdgpu_buffer_rsrc_t b = c.strip(j);
  const uint64_t W = c.W();
#pragma unroll
  for (int r = 0; r < P - 1; ++r) st<VT>(b, r, W, c.col, v[r]);
}

// Q = reduction of acc_q from C to R_p: row r plus row p-1.
template <int P, int V, class C>
__device__ __forceinline__ void store_reduced(const C& c, int j, const typename vec_t<V>::type (&aq)[P]) {
  typedef typename vec_t<V>::type VT;
  const __amdgpu_buffer_rsrc_t b = c.strip(j);
  const uint64_t W = c.W();
  const VT top = aq[P - 1];
#pragma unroll
  for (int r = 0; r < P - 1; ++r) st<VT>(b, r, W, c.col, aq[r] ^ top);
}

// Full encode of one tile: P and Q (either may be skipped).
template <int P, int V, int U, bool EXT, class C>
__device__ __forceinline__ void tile_encode(const C& c, int k, bool wp, bool wq) {
  typedef typename vec_t<V>::type VT;
  VT ap[P - 1], aq[P];
#pragma unroll
  for (int r = 0; r < P - 1; ++r) ap[r] = (VT)(0u);
#pragma unroll
  for (int u = 0; u < P; ++u) aq[u] = (VT)(0u);
  if (wp && wq) {
    stream_data<P, V, U, true, true, EXT>(c, k, -1, -1, ap, aq);
  } else if (wp) {
    stream_data<P, V, U, true, false, EXT>(c, k, -1, -1, ap, aq);
  } else {
    stream_data<P, V, U, false, true, EXT>(c, k, -1, -1, ap, aq);
  }
  if (wp) store_strip<P, V>(c, k, ap);
  if (wq) store_reduced<P, V>(c, k + 1, aq);
}

// Component c of a vector (a dword column of the thread's slice).
template <int V> struct comp;
template <> struct comp<1> {
  static __device__ __forceinline__ uint32_t get(uint32_t v, int) { return v; }
  static __device__ __forceinline__ void set(uint32_t& v, int, uint32_t x) { v = x; }
};
template <int V> struct comp {
  typedef typename vec_t<V>::type VT;
  static __device__ __forceinline__ uint32_t get(const VT& v, int c) { return v[c]; }
  static __device__ __forceinline__ void set(VT& v, int c, uint32_t x) { v[c] = x; }
};

// Solve (1 + x^z) D = T for one dword column held in LDS (rows 0..p-1 of a
// lift T~ of T), in place: the chain described at the top of this file, with
// e the XOR of all p rows of T~.  Afterwards the column holds D~ with
// D~[p-1] = 0, i.e. rows 0..p-2 are D.
template <int P>
__device__ __forceinline__ void chain_solve(uint32_t* lds, int ls, int z, uint32_t e) {
  constexpr int R = P - 1;
  // Rows u_s = (p-1 + s z) mod p, s = 1..p-1; each row is visited once.  The
  // next row's value is read before the current one is written: rows of
  // consecutive steps differ, so the read does not see the write.
  int u = R + z;
  if (u >= P) u -= P;
  uint32_t t = lds[u * ls];
  uint32_t d = 0u;
#pragma unroll
  for (int s = 0; s < R; ++s) {
    int un = u + z;
    if (un >= P) un -= P;
    const uint32_t tn = (s + 1 < R) ? lds[un * ls] : 0u;
    d = t ^ e ^ d;
    lds[u * ls] = d;
    t = tn;
    u = un;
  }
}

// Inverse of f in R_p = F2[x]/(1 + x + ... + x^{p-1}); polynomials are bit
// masks (bit i = coefficient of x^i).  Extended Euclid against
// Phi_p = 1 + x + ... + x^{p-1}, keeping s with s*f = r (mod Phi_p); ends when
// r = 1 and returns s, of degree < p-1.  The arguments are uniform over the
// wave, so this runs on the scalar unit.  Every step lowers deg r, so the
// loops end after at most 64 rounds even for a non-invertible f (which the
// host's checks exclude).
__device__ __forceinline__ uint64_t inverse_mod_phi(uint64_t f, int p) {
  const uint64_t phi = (1ull << p) - 1ull;
  if ((f >> (p - 1)) & 1ull) f ^= phi;
  uint64_t r0 = phi, r1 = f, s0 = 0ull, s1 = 1ull;
  while (r1 > 1ull) {
    const int d1 = 63 - __builtin_clzll(r1);
    int d0 = 63 - __builtin_clzll(r0);
    while (d0 >= d1) {
      r0 ^= r1 << (d0 - d1);
      s0 ^= s1 << (d0 - d1);
      if (r0 == 0ull) break;
      d0 = 63 - __builtin_clzll(r0);
    }
    const uint64_t tr = r0, ts = s0;
    r0 = r1;
    s0 = s1;
    r1 = tr;
    s1 = ts;
  }
  return s1;
}

// Finishing of a recovery from the syndromes of the surviving strips, for
// the cases D, DQ, DP and DD (a thread's V-dword column slice):
//   D, DQ, DD: ap = P + sum of the surviving data strips (dP);
//   DP:        ap = sum of the surviving data strips (P is rebuilt);
//   DP, DD:    aq = Q~ + sum of the surviving g_t D_t, in C (dQ~);
//   DQ:        aq = sum of the surviving g_t D_t, in C (Q is rebuilt).
// `lds` points at this thread's column of a region of P rows of one dword,
// row stride `ls` dwords; only this thread touches it.  The data-dependent
// row permutations are done one dword column at a time, so the region does
// not grow with the vector width.
//
// EXT: the stripe has k > p data strips and the extended Q parity of
// Section 3.3 (coefficient g_t = x^t for t < p, 1 + x^{t-p+1} for t >= p).
// The general recovery formulas of the proof of Lemma 3.1.2 then read
//   data x + P:  g_x D_x = dQ,
//   data x + Q:  D_x = dP, Q = (Q sum without x) + g_x D_x,
//   data x < y:  (g_x + g_y) D_y = g_x dP + dQ,  D_x = D_y + dP,
// with dP, dQ the syndromes of the surviving strips.  g_x + g_y is
// x^x (1 + x^{y-x}) when both are below p, x^i (1 + x^{j-i}) when both are
// extended (i = x-p+1, j = y-p+1), both solved by the chain; for x < p <= y
// it is the trinomial 1 + x^x + x^j, whose inverse h (Theorem 3.3.3 makes it
// exist) is computed per wave and applied as the cyclic convolution
// D~[u] = sum_{i in h} G~[u - i] in C.
template <int P, int V, bool EXT, class C>
__device__ __forceinline__ void finish_recover(const C& c, int k, const Case& cs,
                                               typename vec_t<V>::type (&ap)[P - 1],
                                               typename vec_t<V>::type (&aq)[P], uint32_t* lds, int ls) {
  typedef typename vec_t<V>::type VT;
  typedef comp<V> CP;
  constexpr int R = P - 1;
  const int iP = k, iQ = k + 1;

  if (cs.op == OP_D) {
    // D_x = P + sum_{t != x} D_t.
    store_strip<P, V>(c, cs.x, ap);
    return;
  }

  if (cs.op == OP_DQ) {
    // D_x = dP;  Q = sum_{t != x} g_t D_t + g_x D_x.
    const int x = cs.x;
    const bool xe = EXT && x >= P;        // g_x = 1 + x^{sh}, else x^{sh}
    const int sh = xe ? x - P + 1 : x;
#pragma unroll
    for (int cc = 0; cc < V; ++cc) {
#pragma unroll
      for (int r = 0; r < R; ++r) lds[r * ls] = CP::get(ap[r], cc);
      lds[R * ls] = 0u;
      // (x^sh D~)[u] = D~[(u - sh) mod p]
#pragma unroll
      for (int u = 0; u < P; ++u) {
        int w = u - sh;
        if (w < 0) w += P;
        CP::set(aq[u], cc, CP::get(aq[u], cc) ^ lds[w * ls]);
      }
    }
    if (xe) {
#pragma unroll
      for (int r = 0; r < R; ++r) aq[r] ^= ap[r];
    }
    store_strip<P, V>(c, x, ap);
    store_reduced<P, V>(c, iQ, aq);
    return;
  }

  if (cs.op == OP_DP) {
    // g_x D_x = Q + sum_{t != x} g_t D_t;  P = sum_{t != x} D_t + D_x.
    const int x = cs.x;
    if (EXT && x >= P) {
      // (1 + x^j) D_x = dQ, j = x-p+1: the chain on the lift dQ~.
      const int j = x - P + 1;
#pragma unroll
      for (int cc = 0; cc < V; ++cc) {
        uint32_t e = 0u;
#pragma unroll
        for (int u = 0; u < P; ++u) {
          const uint32_t t = CP::get(aq[u], cc);
          lds[u * ls] = t;
          e ^= t;
        }
        chain_solve<P>(lds, ls, j, e);
#pragma unroll
        for (int r = 0; r < R; ++r) CP::set(aq[r], cc, lds[r * ls]);
      }
      const __amdgpu_buffer_rsrc_t bx = c.strip(x), bp = c.strip(iP);
      const uint64_t W = c.W();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        st<VT>(bx, r, W, c.col, aq[r]);
        st<VT>(bp, r, W, c.col, aq[r] ^ ap[r]);
      }
      return;
    }
    // D_x = x^{p-x} dQ:  (x^{p-x} a)[u] = a[(u + x) mod p], in place.
#pragma unroll
    for (int cc = 0; cc < V; ++cc) {
#pragma unroll
      for (int u = 0; u < P; ++u) lds[u * ls] = CP::get(aq[u], cc);
#pragma unroll
      for (int u = 0; u < P; ++u) {
        int w = u + x;
        if (w >= P) w -= P;
        CP::set(aq[u], cc, lds[w * ls]);
      }
    }
    // Reduce (row r plus row p-1), store D_x, then P = (data sum) + D_x.
    const __amdgpu_buffer_rsrc_t bx = c.strip(x), bp = c.strip(iP);
    const uint64_t W = c.W();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const VT d = aq[r] ^ aq[R];
      st<VT>(bx, r, W, c.col, d);
      st<VT>(bp, r, W, c.col, d ^ ap[r]);
    }
    return;
  }

  // OP_DD: data x < y.
  const int x = cs.x, y = cs.y;

  if (EXT && x < P && y >= P) {
    // (1 + x^x + x^j) D_y = x^x dP + dQ =: G, j = y-p+1.  (x = 0 gives x^j,
    // x = j gives 1; the inverse covers both.)
    const int j = y - P + 1;
    const uint64_t h = inverse_mod_phi((1ull << x) ^ (1ull << j) ^ 1ull, P);
#pragma unroll
    for (int cc = 0; cc < V; ++cc) {
#pragma unroll
      for (int r = 0; r < R; ++r) lds[r * ls] = CP::get(ap[r], cc);
      lds[R * ls] = 0u;
      uint32_t g[P];
#pragma unroll
      for (int u = 0; u < P; ++u) {
        int w = u - x;
        if (w < 0) w += P;
        g[u] = CP::get(aq[u], cc) ^ lds[w * ls];
      }
#pragma unroll
      for (int u = 0; u < P; ++u) lds[u * ls] = g[u];
#pragma unroll
      for (int u = 0; u < P; ++u) g[u] = 0u;
      for (uint64_t m = h; m != 0ull; m &= m - 1ull) {
        const int i = __builtin_ctzll(m) % P;
#pragma unroll
        for (int u = 0; u < P; ++u) {
          int w = u - i;
          if (w < 0) w += P;
          g[u] ^= lds[w * ls];
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) CP::set(aq[r], cc, g[r] ^ g[R]);
    }
  } else {
    // (1 + x^z) D_y = T with T = dP + x^{-s} dQ', where
    //   both below p:    s = x,      z = y - x, dQ' = dQ;
    //   both extended:   s = x-p+1,  z = y - x, dQ' = dQ + dP.
    const bool both_ext = EXT && x >= P;
    const int s = both_ext ? x - P + 1 : x;
    const int z = y - x;
    if (both_ext) {
#pragma unroll
      for (int r = 0; r < R; ++r) aq[r] ^= ap[r];
    }
#pragma unroll
    for (int cc = 0; cc < V; ++cc) {
      // T~[u] = dP~[u] + dQ'~[(u + s) mod p], built in aq (natural row order).
#pragma unroll
      for (int u = 0; u < P; ++u) lds[u * ls] = CP::get(aq[u], cc);
      uint32_t e = 0u;  // XOR of all p rows of T~
#pragma unroll
      for (int u = 0; u < P; ++u) {
        int w = u + s;
        if (w >= P) w -= P;
        uint32_t t = lds[w * ls];
        if (u < R) t ^= CP::get(ap[u], cc);
        e ^= t;
        CP::set(aq[u], cc, t);
      }
#pragma unroll
      for (int u = 0; u < P; ++u) lds[u * ls] = CP::get(aq[u], cc);
      chain_solve<P>(lds, ls, z, e);
      // D_y in natural row order back into aq.
#pragma unroll
      for (int r = 0; r < R; ++r) CP::set(aq[r], cc, lds[r * ls]);
    }
  }
  const __amdgpu_buffer_rsrc_t bx = c.strip(x), by = c.strip(y);
  const uint64_t W = c.W();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    st<VT>(by, r, W, c.col, aq[r]);
    st<VT>(bx, r, W, c.col, aq[r] ^ ap[r]);
  }
}

// Recovery of one tile by one thread's V-dword column slice: the streaming
// phase for the case, then finish_recover.  `lds`, `ls` as there.
template <int P, int V, int U, bool EXT, class C>
__device__ __forceinline__ void tile_recover(const C& c, int k, const Case& cs_in, uint32_t* lds, int ls) {
  typedef typename vec_t<V>::type VT;
  constexpr int R = P - 1;
  const int iP = k, iQ = k + 1;
  // The case is uniform over the wave; keep it (and every strip address
  // derived from it) in scalar registers.
  const Case cs{__builtin_amdgcn_readfirstlane(cs_in.op), __builtin_amdgcn_readfirstlane(cs_in.x),
                __builtin_amdgcn_readfirstlane(cs_in.y)};

  switch (cs.op) {
    case OP_PQ:
      tile_encode<P, V, U, EXT>(c, k, true, true);
      return;
    case OP_P:
      tile_encode<P, V, U, EXT>(c, k, true, false);
      return;
    case OP_Q:
      tile_encode<P, V, U, EXT>(c, k, false, true);
      return;
    default:
      break;
  }

  VT ap[R], aq[P];
#pragma unroll
  for (int u = 0; u < P; ++u) aq[u] = (VT)(0u);

  // dP with P itself in ap (cases D, DQ, DD).  With extended parity acc_p
  // must start at zero, so P comes last there.
  auto with_p = [&](int y) {
    if constexpr (EXT) {
#pragma unroll
      for (int r = 0; r < R; ++r) ap[r] = (VT)(0u);
      stream_data<P, V, U, true, true, true>(c, k, cs.x, y, ap, aq);
      xor_from<P, V>(c, iP, ap);
    } else {
      load_into<P, V>(c, iP, ap);
      stream_data<P, V, U, true, true, false>(c, k, cs.x, y, ap, aq);
    }
  };
  // Each case keeps its own streaming code and finishing, so that the
  // compiler allocates registers per case.
  if (cs.op == OP_D) {
    load_into<P, V>(c, iP, ap);
    stream_range<P, V, U, true, false>(c, k - 1, 0, cs.x, -1, ap, aq);
    finish_recover<P, V, EXT>(c, k, Case{OP_D, cs.x, -1}, ap, aq, lds, ls);
  } else if (cs.op == OP_DP) {
#pragma unroll
    for (int r = 0; r < R; ++r) ap[r] = (VT)(0u);
    stream_data<P, V, U, true, true, EXT>(c, k, cs.x, -1, ap, aq);
    xor_from<P, V>(c, iQ, aq);
    finish_recover<P, V, EXT>(c, k, Case{OP_DP, cs.x, -1}, ap, aq, lds, ls);
  } else if (cs.op == OP_DQ) {
    with_p(-1);
    finish_recover<P, V, EXT>(c, k, Case{OP_DQ, cs.x, -1}, ap, aq, lds, ls);
  } else {
    with_p(cs.y);
    xor_from<P, V>(c, iQ, aq);
    finish_recover<P, V, EXT>(c, k, Case{OP_DD, cs.x, cs.y}, ap, aq, lds, ls);
  }
}

// Recovery of one tile with one streaming pass for every case (same
// arguments and results as tile_recover).  The kernel then holds one copy of
// the unrolled loop instead of one per case: the job-list kernel (two load
// policies, every case) shrinks from 66-186 KB to 23-61 KB at the same
// speed.  The strided kernels keep tile_recover's per-case loops, which
// measured faster there (p = 29 double-data recovery 78% vs 72% of peak).
//  * PQ, P, Q (re-encode): nothing erased is skipped, P and Q start at 0;
//  * D, DQ, DD: P itself enters acc_p (plain code: first; extended: after
//    the pass, which needs acc_p to start at zero);
//  * DP, DD: Q itself enters acc_q after the pass.
template <int P, int V, int U, bool EXT, class C>
__device__ __forceinline__ void tile_recover_one_pass(const C& c, int k, const Case& cs_in, uint32_t* lds,
                                                      int ls) {
  typedef typename vec_t<V>::type VT;
  constexpr int R = P - 1;
  const int iP = k, iQ = k + 1;
  const Case cs{__builtin_amdgcn_readfirstlane(cs_in.op), __builtin_amdgcn_readfirstlane(cs_in.x),
                __builtin_amdgcn_readfirstlane(cs_in.y)};
  const bool enc = cs.op == OP_PQ || cs.op == OP_P || cs.op == OP_Q;
  const bool with_p = cs.op == OP_D || cs.op == OP_DQ || cs.op == OP_DD;
  const bool with_q = cs.op == OP_DP || cs.op == OP_DD;
  VT ap[R], aq[P];
#pragma unroll
  for (int u = 0; u < P; ++u) aq[u] = (VT)(0u);
  if (!EXT && with_p) {
    load_into<P, V>(c, iP, ap);
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) ap[r] = (VT)(0u);
  }
  stream_data<P, V, U, true, true, EXT>(c, k, enc ? -1 : cs.x, cs.op == OP_DD ? cs.y : -1, ap, aq);
  if (EXT && with_p) xor_from<P, V>(c, iP, ap);
  if (with_q) xor_from<P, V>(c, iQ, aq);
  if (enc) {
    if (cs.op != OP_Q) store_strip<P, V>(c, k, ap);
    if (cs.op != OP_P) store_reduced<P, V>(c, k + 1, aq);
    return;
  }
  finish_recover<P, V, EXT>(c, k, cs, ap, aq, lds, ls);
}

// Split-K tile (plain code; EXT: extended Q parity, see below).  The S waves of the work-group share one column
// tile of 64 lanes x V dwords starting at byte `tile_base` of a row (this
// thread's slice is c.col) and split the data strips into S contiguous
// ranges [t0, t1); each wave runs the streaming phase on its range.  Its Q
// partial is x^{t0} times what Horner leaves (sum_t x^{t-t0} D_t), so it goes
// to LDS rotated by t0, next to the P partial; wave 0 (whose range starts at
// t = 0) also adds P and/or Q where the case needs them.  After a barrier:
//  * encode-like cases: the waves split the rows, sum the S partials and
//    store P and the reduced Q (row r plus row p-1) V dwords per lane;
//  * recoveries: one thread per dword column sums its column of the
//    partials and runs finish_recover on it, with its LDS column as the
//    permutation scratch.
// Many waves on one stripe at a time keeps fewer stripes in flight, which
// the memory system rewards.  `part` holds S*(2p-1)*64*V dwords; the case
// must be uniform over the work-group and every thread must call this.
template <int P, int V, int U, int S, bool EXT, class C>
__device__ __forceinline__ void tile_split(const C& c, int k, const Case& cs_in, uint32_t tile_base,
                                           uint32_t* part) {
  typedef typename vec_t<V>::type VT;
  typedef comp<V> CP;
  constexpr int R = P - 1;
  constexpr int NR = 2 * P - 1;
  constexpr int CS = 64 * V;                  // dword columns of the tile
  const Case cs{__builtin_amdgcn_readfirstlane(cs_in.op), __builtin_amdgcn_readfirstlane(cs_in.x),
                __builtin_amdgcn_readfirstlane(cs_in.y)};
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const uint32_t col = c.col;
  const bool live = col < c.W();
  // Erased data strips are skipped; P/Q are rebuilt, never read, in their cases.
  const int x = (cs.op == OP_D || cs.op == OP_DP || cs.op == OP_DQ || cs.op == OP_DD) ? cs.x : -1;
  const int y = cs.op == OP_DD ? cs.y : -1;
  const bool add_p = cs.op == OP_D || cs.op == OP_DQ || cs.op == OP_DD;
  const bool add_q = cs.op == OP_DP || cs.op == OP_DD;
  // Balanced contiguous ranges: the strips a wave loads (surviving data
  // strips, and for wave 0 also P and/or Q) are split evenly.  pos(m) is the
  // first t with m surviving data strips below it.
  const int surv = k - (x >= 0) - (y >= 0);
  const int extra = (int)add_p + (int)add_q;
  const int per = (surv + extra + S - 1) / S;
  auto pos = [&](int m) {
    int t = m;
    if (x >= 0 && x < t) ++t;
    if (y >= 0 && y < t) ++t;
    return t;
  };
  auto clampm = [&](int m) { return m < 0 ? 0 : (m > surv ? surv : m); };
  const int t0 = pos(clampm(w * per - extra));
  const int t1 = pos(clampm((w + 1) * per - extra));
  VT ap[R], aq[P];
#pragma unroll
  for (int r = 0; r < R; ++r) ap[r] = (VT)(0u);
#pragma unroll
  for (int u = 0; u < P; ++u) aq[u] = (VT)(0u);
  // Extended Q parity (Section 3.3): in C, strip t >= p enters Q with
  // 1 + x^{t+1}.  A range that straddles p takes the transition of
  // stream_data at t = p: acc_q <- x acc_q + acc_p, where acc_p then holds
  // exactly the strips >= p.  A range entirely above p multiplies its Horner
  // sum by x once, and its plain sum (its P partial) joins the Q partial
  // unrotated (below).
  bool above_p = false;
  if (live) {
    if (t0 < t1) {
      if (!EXT || t1 <= P) {
        stream_range<P, V, U, true, true>(c, t1 - 1, t0, x, y, ap, aq);
      } else if (t0 < P) {
        stream_range<P, V, U, true, true>(c, t1 - 1, P, x, y, ap, aq);
        rotate_up<P>(aq);
#pragma unroll
        for (int r = 0; r < R; ++r) aq[r] ^= ap[r];
        stream_range<P, V, U, true, true>(c, P - 1, t0, x, y, ap, aq);
      } else {
        stream_range<P, V, U, true, true>(c, t1 - 1, t0, x, y, ap, aq);
        rotate_up<P>(aq);
        above_p = true;
      }
    }
    if (w == 0) {   // t0 = 0 here, so Q enters unrotated
      if (add_p) xor_from<P, V>(c, k, ap);
      if (add_q) xor_from<P, V>(c, k + 1, aq);
    }
  }
  uint32_t* my = part + (size_t)w * NR * CS + lane * V;
  const int rot = t0 % P;
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < V; ++j) my[r * CS + j] = CP::get(ap[r], j);
#pragma unroll
  for (int u = 0; u < P; ++u) {
    int d = u + rot;
    if (d >= P) d -= P;
#pragma unroll
    for (int j = 0; j < V; ++j) my[(R + d) * CS + j] = CP::get(aq[u], j);
  }
  if (EXT && above_p) {
    // Only this thread touches these LDS words: no barrier needed before.
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < V; ++j) my[(R + r) * CS + j] ^= CP::get(ap[r], j);
  }
  __syncthreads();

  if (cs.op == OP_PQ || cs.op == OP_P || cs.op == OP_Q) {
    if (!live) return;
    auto row = [&](int rr) {
      VT v = (VT)(0u);
#pragma unroll
      for (int s2 = 0; s2 < S; ++s2)
#pragma unroll
        for (int j = 0; j < V; ++j)
          CP::set(v, j, CP::get(v, j) ^ part[((size_t)s2 * NR + rr) * CS + lane * V + j]);
      return v;
    };
    const VT top = row(R + R);
    const __amdgpu_buffer_rsrc_t bp = c.strip(k), bq = c.strip(k + 1);
    const uint64_t W = c.W();
    for (int r = w; r < R; r += S) {
      if (cs.op != OP_Q) st<VT>(bp, r, W, col, row(r));
      if (cs.op != OP_P) st<VT>(bq, r, W, col, row(R + r) ^ top);
    }
    return;
  }

  for (int cc = threadIdx.x; cc < CS; cc += 64 * S) {
    const uint32_t cb = tile_base + (uint32_t)cc * 4u;
    if (cb >= c.W()) break;
    uint32_t fp[R], fq[P];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      uint32_t v = 0u;
#pragma unroll
      for (int s2 = 0; s2 < S; ++s2) v ^= part[((size_t)s2 * NR + r) * CS + cc];
      fp[r] = v;
    }
#pragma unroll
    for (int u = 0; u < P; ++u) {
      uint32_t v = 0u;
#pragma unroll
      for (int s2 = 0; s2 < S; ++s2) v ^= part[((size_t)s2 * NR + R + u) * CS + cc];
      fq[u] = v;
    }
    // Only this thread uses column cc of the partials from here on.
    C cd = c;
    cd.col = cb;
    finish_recover<P, 1, EXT>(cd, k, cs, fp, fq, part + cc, CS);
  }
}

}  // namespace raid6c
