// layout.hip -- interop with the horizontal Z_17 layout of Section 4.5.
//
// There a strip is an array of 16-bit words, one codeword of R_17 each, bit
// r being the coefficient of x^r.  Here a strip is 16 rows of W bytes and the
// codeword of lane (byte j, bit b) has its x^r coefficient in bit b of byte j
// of row r; codeword c of a horizontal strip (8W words) is lane (c/8, c%8).
// Both layouts hold the same ring elements, so converting, encoding here and
// converting back gives the parity the paper's routine computes.
//
// Each thread converts 32 consecutive codewords (64 bytes) <-> one dword of
// each of the 16 rows: a 16 x 32 bit-matrix transpose in registers, done as
// two 16 x 16 transposes side by side in the halves of 16 dwords (four
// butterfly stages of masked swaps).  The vertical side is dword rows,
// contiguous across the lanes of a wave.  On the horizontal side each thread
// loads its 64 bytes directly (four 16-byte loads, which the caches serve
// well), but stores go through LDS: the work-group's 256 x 64 bytes leave
// LDS in 16-byte vectors contiguous across the lanes, so no store
// instruction spans more than the bytes it writes (direct stores of each
// thread's 64 bytes ran at 63% of the HBM peak, these at 72%).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "raid6c_internal.h"

namespace raid6c {

namespace {

// a[i] holds the bits of two 16 x 16 blocks (low and high halves).  After the
// call, bit c of half h of a[r] is bit r of half h of the input a[c]; the map
// is its own inverse.
__device__ __forceinline__ void transpose16x2(uint32_t (&a)[16]) {
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int s = 8 >> st;
    const uint32_t m = st == 0 ? 0x00FF00FFu : st == 1 ? 0x0F0F0F0Fu : st == 2 ? 0x33333333u : 0x55555555u;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if (i & s) continue;
      const uint32_t t = ((a[i] >> s) ^ a[i + s]) & m;
      a[i + s] ^= t;
      a[i] ^= t << s;
    }
  }
}

constexpr int kZ17Threads = 256;

// LDS slot of 16-byte vector i of a work-group's 256 x 64 bytes.  Thread t
// writes vectors 4t..4t+3; rotating the low three bits of the slot by bits
// 3..5 puts the vectors that 8 neighbouring threads write at once in 8
// different 16-byte bank groups.  Consecutive vectors (the HBM side) stay
// within one aligned group of 8 slots.
__device__ __forceinline__ uint32_t z17_slot(uint32_t i) { return (i & ~7u) | ((i + (i >> 3)) & 7u); }

__global__ void __launch_bounds__(kZ17Threads) z17_to_vertical_kernel(const uint4* words, uint32_t* strips,
                                                                       uint64_t cols, uint64_t total) {
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const uint64_t s = g / cols, j = g - s * cols;
  const uint4* in = words + g * 4;                 // 32 codewords = 64 bytes
  const uint4 q0 = in[0], q1 = in[1], q2 = in[2], q3 = in[3];
  const uint32_t d[16] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w,
                          q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w};
  // a[i] = word i | word 16+i << 16 (word 2m is the low half of d[m]).
  uint32_t a[16];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    a[2 * m] = (d[m] & 0xFFFFu) | (d[8 + m] << 16);
    a[2 * m + 1] = (d[m] >> 16) | (d[8 + m] & 0xFFFF0000u);
  }
  transpose16x2(a);
  uint32_t* out = strips + s * 16 * cols + j;
#pragma unroll
  for (int r = 0; r < 16; ++r) out[r * cols] = a[r];
}

__global__ void __launch_bounds__(kZ17Threads) z17_to_horizontal_kernel(const uint32_t* strips, uint4* words,
                                                                         uint64_t cols, uint64_t total) {
  __shared__ uint4 stage[kZ17Threads * 4];
  const uint64_t g0 = (uint64_t)blockIdx.x * kZ17Threads;
  const uint32_t nvec = (uint32_t)((total - g0 < kZ17Threads ? total - g0 : kZ17Threads) * 4);
  const uint64_t g = g0 + threadIdx.x;
  if (g < total) {
    const uint64_t s = g / cols, j = g - s * cols;
    const uint32_t* in = strips + s * 16 * cols + j;
    uint32_t a[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) a[r] = in[r * cols];
    transpose16x2(a);
    uint32_t d[16];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      d[m] = (a[2 * m] & 0xFFFFu) | (a[2 * m + 1] << 16);
      d[8 + m] = (a[2 * m] >> 16) | (a[2 * m + 1] & 0xFFFF0000u);
    }
    const uint32_t v = threadIdx.x * 4;
    stage[z17_slot(v)] = uint4{d[0], d[1], d[2], d[3]};
    stage[z17_slot(v + 1)] = uint4{d[4], d[5], d[6], d[7]};
    stage[z17_slot(v + 2)] = uint4{d[8], d[9], d[10], d[11]};
    stage[z17_slot(v + 3)] = uint4{d[12], d[13], d[14], d[15]};
  }
  __syncthreads();
  uint4* dst = words + g0 * 4;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const uint32_t i = m * kZ17Threads + threadIdx.x;
    if (i < nvec) dst[i] = stage[z17_slot(i)];
  }
}

}  // namespace

hipError_t z17_launch(bool to_vertical, const void* in, void* out, uint64_t row_bytes, uint64_t count,
                      hipStream_t stream) {
  const uint64_t cols = row_bytes / 4;
  const uint64_t total = cols * count;
  const int threads = kZ17Threads;
  const uint64_t blocks = (total + threads - 1) / threads;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  if (to_vertical)
    hipLaunchKernelGGL(z17_to_vertical_kernel, dim3((uint32_t)blocks), dim3(threads), 0, stream,
                       (const uint4*)in, (uint32_t*)out, cols, total);
  else
    hipLaunchKernelGGL(z17_to_horizontal_kernel, dim3((uint32_t)blocks), dim3(threads), 0, stream,
                       (const uint32_t*)in, (uint4*)out, cols, total);
  return hipGetLastError();
}

}  // namespace raid6c
