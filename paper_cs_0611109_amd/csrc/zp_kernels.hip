// zp_kernels.hip -- Z_p-RAID encode and recovery kernels for one prime.
//
// This file is compiled twice per supported prime, with -DRAID6C_P=<p> and
// -DRAID6C_EXT=0 or 1: the plain code (k <= p) and the extended Q parity
// (p < k <= 2p-1, Section 3.3) go to separate objects, so that the code of
// one never shapes the compiler's choices for the other.  Each pair of
// objects contributes one entry to the dispatch table of the host API.
//
// Grid: one work-group per (stripe, column tile); a tile is `threads` threads
// times V dwords of every row.  Work-group i handles stripe i / tiles and tile
// i % tiles, so the stripe and its erasure case are uniform over the group and
// all strip addresses live in scalar registers.
#ifndef RAID6C_EXT
#define RAID6C_EXT 0
#endif
#define RAID6C_UNIFORM_ROW_HINT RAID6C_EXT
#include "zp_core.hpp"

#ifndef RAID6C_P
#error "compile with -DRAID6C_P=<odd prime>"
#endif

#define RAID6C_CAT2(a, b) a##b
#define RAID6C_CAT(a, b) RAID6C_CAT2(a, b)

namespace raid6c {

namespace {

constexpr int kP = RAID6C_P;
constexpr bool kExt = RAID6C_EXT != 0;
static_assert(kP >= 3 && kP <= kMaxPrime && (kP % 2) == 1, "unsupported prime");

// Vector widths built for this prime: wider vectors need (2p-1)*V registers
// for the two accumulators, so they are only built for small p.
constexpr int kVecMask = (kP <= 13) ? (1 | 2 | 4) : (kP <= 31) ? (1 | 2) : 1;

// EXT: k > p data strips with the extended Q parity of Section 3.3.
template <int P, int V, int U, bool EXT>
__global__ void __launch_bounds__(256) zp_encode_kernel(const ZpArgs a) {
  const uint32_t stripe = blockIdx.x / a.tiles;
  const uint32_t tile = blockIdx.x - stripe * a.tiles;
  const uint32_t col = (tile * blockDim.x + threadIdx.x) * (V * 4);
  if (col >= a.row_bytes) return;
  const ColsTable c{&a, (uint64_t)stripe * a.stripe_stride, (uint64_t)stripe * a.src_stripe_stride, col,
                    (uint32_t)((P - 1) * a.row_bytes)};
  tile_encode<P, V, U, EXT>(c, a.k, true, true);
}

template <int P, int V, int U, bool EXT>
__global__ void __launch_bounds__(256) zp_recover_kernel(const ZpArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const uint32_t stripe = blockIdx.x / a.tiles;
  const uint32_t tile = blockIdx.x - stripe * a.tiles;
  int e0 = a.e0, e1 = a.e1;
  if (a.erasures != nullptr) {
    // One stripe per work-group: the entry is uniform.  Saying so keeps the
    // strip addresses derived from it in scalar registers.
    e0 = __builtin_amdgcn_readfirstlane(a.erasures[2 * (uint64_t)stripe]);
    e1 = __builtin_amdgcn_readfirstlane(a.erasures[2 * (uint64_t)stripe + 1]);
  }
  const Case cs = classify(a.k, e0, e1);
  if (cs.op == OP_BAD) {
    if (tile == 0 && threadIdx.x == 0 && a.bad_count != nullptr) atomicAdd(a.bad_count, 1);
    return;
  }
  const uint32_t col = (tile * blockDim.x + threadIdx.x) * (V * 4);
  if (col >= a.row_bytes) return;
  const ColsTable c{&a, (uint64_t)stripe * a.stripe_stride, 0, col, (uint32_t)((P - 1) * a.row_bytes)};
  uint32_t* lds = reinterpret_cast<uint32_t*>(smem) + threadIdx.x;
  tile_recover<P, V, U, EXT>(c, a.k, cs, lds, (int)blockDim.x);
}

// (vec, unroll) pairs built for this prime: accumulators take (2p-1)*vec
// dwords per thread and a batch of loads unroll*(p-1)*vec more.
template <int V, int U>
constexpr bool built() {
  return (kVecMask & V) != 0 && (2 * kP - 1) * V + U * (kP - 1) * V <= 192;
}

constexpr int unroll_mask(int v) {
  return v == 1 ? ((built<1, 1>() ? 1 : 0) | (built<1, 2>() ? 2 : 0) | (built<1, 4>() ? 4 : 0))
       : v == 2 ? ((built<2, 1>() ? 1 : 0) | (built<2, 2>() ? 2 : 0) | (built<2, 4>() ? 4 : 0))
       : v == 4 ? ((built<4, 1>() ? 1 : 0) | (built<4, 2>() ? 2 : 0) | (built<4, 4>() ? 4 : 0))
                : 0;
}

template <int V, int U>
hipError_t launch_vu(ZpKind kind, const ZpConfig& cfg, const ZpArgs& a, uint32_t grid,
                     hipStream_t stream) {
  if constexpr (built<V, U>()) {
    const dim3 g(grid), b(cfg.threads);
    const size_t lds = (size_t)kP * cfg.threads * 4;
    if ((a.k > kP) != kExt) return hipErrorInvalidValue;
    if (kind == KIND_ENCODE) hipLaunchKernelGGL((zp_encode_kernel<kP, V, U, kExt>), g, b, 0, stream, a);
    else hipLaunchKernelGGL((zp_recover_kernel<kP, V, U, kExt>), g, b, lds, stream, a);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

hipError_t launch(ZpKind kind, const ZpConfig& cfg, const ZpArgs& a, uint32_t grid,
                  hipStream_t stream) {
  switch (cfg.vec * 8 + cfg.unroll) {
    case 9: return launch_vu<1, 1>(kind, cfg, a, grid, stream);
    case 10: return launch_vu<1, 2>(kind, cfg, a, grid, stream);
    case 12: return launch_vu<1, 4>(kind, cfg, a, grid, stream);
    case 17: return launch_vu<2, 1>(kind, cfg, a, grid, stream);
    case 18: return launch_vu<2, 2>(kind, cfg, a, grid, stream);
    case 20: return launch_vu<2, 4>(kind, cfg, a, grid, stream);
    case 33: return launch_vu<4, 1>(kind, cfg, a, grid, stream);
    case 34: return launch_vu<4, 2>(kind, cfg, a, grid, stream);
    case 36: return launch_vu<4, 4>(kind, cfg, a, grid, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

#if RAID6C_EXT
hipError_t RAID6C_CAT(zp_launch_ext_, RAID6C_P)(ZpKind kind, const ZpConfig& cfg, const ZpArgs& a, uint32_t grid,
                                                hipStream_t stream) {
  return launch(kind, cfg, a, grid, stream);
}
#else
hipError_t RAID6C_CAT(zp_launch_ext_, RAID6C_P)(ZpKind kind, const ZpConfig& cfg, const ZpArgs& a, uint32_t grid,
                                                hipStream_t stream);

const ZpPrimeEntry* RAID6C_CAT(zp_entry_, RAID6C_P)() {
  static const ZpPrimeEntry e{kP, &launch, &RAID6C_CAT(zp_launch_ext_, RAID6C_P), kVecMask,
                              {0, unroll_mask(1), unroll_mask(2), 0, unroll_mask(4)}};
  return &e;
}
#endif

}  // namespace raid6c
