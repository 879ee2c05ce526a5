// zp_kernels.hip -- Z_p-RAID encode and recovery kernels for one prime.
//
// This file is compiled once per supported prime with -DRAID6C_P=<p>; each
// object contributes one launcher to the dispatch table of the host API.
//
// Grid: one work-group per (stripe, column tile); a tile is `threads` threads
// times V dwords of every row.  Work-group i handles stripe i / tiles and tile
// i % tiles, so the stripe and its erasure case are uniform over the group and
// all strip addresses live in scalar registers.
#include "zp_core.hpp"

#ifndef RAID6C_P
#error "compile with -DRAID6C_P=<odd prime>"
#endif

#define RAID6C_CAT2(a, b) a##b
#define RAID6C_CAT(a, b) RAID6C_CAT2(a, b)

namespace raid6c {

namespace {

constexpr int kP = RAID6C_P;
static_assert(kP >= 3 && kP <= kMaxPrime && (kP % 2) == 1, "unsupported prime");

// Vector widths built for this prime: wider vectors need (2p-1)*V registers
// for the two accumulators, so they are only built for small p.
constexpr int kVecMask = (kP <= 13) ? (1 | 2 | 4) : (kP <= 31) ? (1 | 2) : 1;

template <int P, int V>
__global__ void __launch_bounds__(256) zp_encode_kernel(const ZpArgs a) {
  const uint32_t stripe = blockIdx.x / a.tiles;
  const uint32_t tile = blockIdx.x - stripe * a.tiles;
  const uint32_t col = (tile * blockDim.x + threadIdx.x) * (V * 4);
  if (col >= a.row_bytes) return;
  const Cols c{&a, (uint64_t)stripe * a.stripe_stride, col, (uint32_t)((P - 1) * a.row_bytes)};
  tile_encode<P, V>(c, a.k, true, true);
}

template <int P, int V>
__global__ void __launch_bounds__(256) zp_recover_kernel(const ZpArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  typedef typename vec_t<V>::type VT;
  const uint32_t stripe = blockIdx.x / a.tiles;
  const uint32_t tile = blockIdx.x - stripe * a.tiles;
  int e0 = a.e0, e1 = a.e1;
  if (a.erasures != nullptr) {
    e0 = a.erasures[2 * (uint64_t)stripe];
    e1 = a.erasures[2 * (uint64_t)stripe + 1];
  }
  const Case cs = classify(a.k, e0, e1);
  if (cs.op == OP_BAD) {
    if (tile == 0 && threadIdx.x == 0 && a.bad_count != nullptr) atomicAdd(a.bad_count, 1);
    return;
  }
  const uint32_t col = (tile * blockDim.x + threadIdx.x) * (V * 4);
  if (col >= a.row_bytes) return;
  const Cols c{&a, (uint64_t)stripe * a.stripe_stride, col, (uint32_t)((P - 1) * a.row_bytes)};
  VT* lds = reinterpret_cast<VT*>(smem) + threadIdx.x;
  tile_recover<P, V>(c, a.k, cs, lds, (int)blockDim.x);
}

template <int V>
hipError_t launch_v(ZpKind kind, const ZpConfig& cfg, const ZpArgs& a, uint32_t grid,
                    hipStream_t stream) {
  const dim3 g(grid), b(cfg.threads);
  if (kind == KIND_ENCODE) {
    hipLaunchKernelGGL((zp_encode_kernel<kP, V>), g, b, 0, stream, a);
  } else {
    const size_t lds = (size_t)kP * cfg.threads * V * 4;
    hipLaunchKernelGGL((zp_recover_kernel<kP, V>), g, b, lds, stream, a);
  }
  return hipGetLastError();
}

hipError_t launch(ZpKind kind, const ZpConfig& cfg, const ZpArgs& a, uint32_t grid,
                  hipStream_t stream) {
  switch (cfg.vec) {
    case 1:
      return launch_v<1>(kind, cfg, a, grid, stream);
#if RAID6C_P <= 31
    case 2:
      return launch_v<2>(kind, cfg, a, grid, stream);
#endif
#if RAID6C_P <= 13
    case 4:
      return launch_v<4>(kind, cfg, a, grid, stream);
#endif
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

const ZpPrimeEntry* RAID6C_CAT(zp_entry_, RAID6C_P)() {
  static const ZpPrimeEntry e{kP, &launch, kVecMask};
  return &e;
}

}  // namespace raid6c
