// zp_kernels.hip -- Z_p-RAID encode and recovery kernels for one prime.
//
// This file is compiled six times per supported prime, with
// -DRAID6C_P=<p> and -DRAID6C_VARIANT=
//   0  the plain code (k <= p), one column slice per thread;
//   1  the extended Q parity (p < k <= 2p-1, Section 3.3), same mapping;
//   2  split-K, plain code and extended Q parity: the waves of a work-group
//      share a column tile and split the data strips;
//   3  the job-list kernel of plans: the tiles of many stripes of this prime,
//      each with its own geometry, one per wave;
//   4  the same for stripes with the extended Q parity (p < k <= 2p-1);
//   5  the job-list kernel for small batches of the request server, set for
//      the latency of one tile rather than for bandwidth: the waves of a
//      work-group share one tile and split its strips.
// Each object is compiled alone so that the code of one never shapes the
// compiler's choices for the others; object 0 holds the dispatch entry and
// calls into the others.
//
// Grid (variants 0, 1): one work-group per (stripe, column tile); a tile is
// `threads` threads times V dwords of every row.  Work-group i handles stripe
// i / tiles and tile i % tiles, so the stripe and its erasure case are uniform
// over the group and all strip addresses live in scalar registers.  Variant
// 2: the same with a tile of 64 lanes times V dwords.
#ifndef RAID6C_VARIANT
#define RAID6C_VARIANT 0
#endif
#define RAID6C_UNIFORM_ROW_HINT (RAID6C_VARIANT != 0)
#include "zp_core.hpp"

#ifndef RAID6C_P
#error "compile with -DRAID6C_P=<odd prime>"
#endif

#define RAID6C_CAT2(a, b) a##b
#define RAID6C_CAT(a, b) RAID6C_CAT2(a, b)

namespace raid6c {

namespace {

constexpr int kP = RAID6C_P;
constexpr bool kExt = RAID6C_VARIANT == 1;
constexpr int sk_lds_bytes_any(int V, int S) { return S * (2 * kP - 1) * 64 * V * 4; }
static_assert(kP >= 3 && kP <= kMaxPrime && (kP % 2) == 1, "unsupported prime");

// Vector widths built for this prime: wider vectors need (2p-1)*V registers
// for the two accumulators; vec 4 only up to p = 13.  Vec 2 for the large
// primes runs at one wave per SIMD with one strip per batch, and on rows that
// are a multiple of its tile it beat vec 1 by 2-6 points of peak.
constexpr int kVecMask = (kP <= 13) ? (1 | 2 | 4) : (1 | 2);

// Work-group order 2: the stripes of consecutive work-groups are spread over
// the launch, stripe s -> s * m mod n with gcd(m, n) = 1 (a permutation), so
// that the work-groups in flight at one time do not all touch the same
// offsets of neighbouring stripes.
__device__ __forceinline__ uint32_t scatter_stripe(uint32_t s, const ZpArgs& a) {
  return a.stripe_mult == 0u ? s : (uint32_t)(((uint64_t)s * a.stripe_mult) % a.nstripes);
}

// EXT: k > p data strips with the extended Q parity of Section 3.3.  LP: cache
// policy of the loads (non-temporal, or the ordinary one when rows do not all
// start on 128-byte lines, whose edge lines two tiles read).  The work-group
// order (dispatch order, or XCD-chunked: xcd_chunk) is a launch parameter;
// launches whose rows are off the lines always take the chunked one.
template <int P, int V, int U, bool EXT, int LP>
__global__ void __launch_bounds__(256) zp_encode_kernel(const ZpArgs a) {
  const uint32_t bid = a.xcd_order ? xcd_chunk(blockIdx.x, gridDim.x) : blockIdx.x;
  const uint32_t tile = bid % a.tiles;
  const uint32_t stripe = scatter_stripe(bid / a.tiles, a);
  const uint32_t col = (tile * blockDim.x + threadIdx.x) * (V * 4);
  if (col >= a.row_bytes) return;
  const ColsTableP<LP> c{&a, (uint64_t)stripe * a.stripe_stride, (uint64_t)stripe * a.src_stripe_stride, col,
                         (uint32_t)((P - 1) * a.row_bytes)};
  tile_encode<P, V, U, EXT>(c, a.k, true, true);
}

template <int P, int V, int U, bool EXT, int LP>
__global__ void __launch_bounds__(256) zp_recover_kernel(const ZpArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const uint32_t bid = a.xcd_order ? xcd_chunk(blockIdx.x, gridDim.x) : blockIdx.x;
  const uint32_t tile = bid % a.tiles;
  const uint32_t stripe = scatter_stripe(bid / a.tiles, a);
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
  const ColsTableP<LP> c{&a, (uint64_t)stripe * a.stripe_stride, 0, col, (uint32_t)((P - 1) * a.row_bytes)};
  uint32_t* lds = reinterpret_cast<uint32_t*>(smem) + threadIdx.x;
  tile_recover<P, V, U, EXT>(c, a.k, cs, lds, (int)blockDim.x);
}

#if RAID6C_VARIANT == 2
// Split-K: the S waves of a work-group share one column tile of one stripe
// and split its data strips (tile_split); EXT: extended Q parity.
template <int P, int V, int U, int S, bool EXT, int LP>
__global__ void __launch_bounds__(64 * S) zp_split_kernel(const ZpArgs a) {
  extern __shared__ __align__(16) uint32_t part[];
  const uint32_t bid = a.xcd_order ? xcd_chunk(blockIdx.x, gridDim.x) : blockIdx.x;
  const uint32_t tile = bid % a.tiles;
  const uint32_t stripe = scatter_stripe(bid / a.tiles, a);
  Case cs{OP_PQ, -1, -1};            // an encode writes P and Q
  if (a.kind == KIND_RECOVER) {
    // Per-stripe entries, or the uniform pair of a single-stripe call.
    int e0 = a.e0, e1 = a.e1;
    if (a.erasures != nullptr) {
      e0 = __builtin_amdgcn_readfirstlane(a.erasures[2 * (uint64_t)stripe]);
      e1 = __builtin_amdgcn_readfirstlane(a.erasures[2 * (uint64_t)stripe + 1]);
    }
    cs = classify(a.k, e0, e1);
    if (cs.op == OP_BAD) {   // uniform over the work-group: no barrier is skipped
      if (tile == 0 && threadIdx.x == 0 && a.bad_count != nullptr) atomicAdd(a.bad_count, 1);
      return;
    }
  }
  const uint32_t col = (tile * 64 + (threadIdx.x & 63)) * (V * 4);
  const ColsTableP<LP> c{&a, (uint64_t)stripe * a.stripe_stride, (uint64_t)stripe * a.src_stripe_stride, col,
                         (uint32_t)((P - 1) * a.row_bytes)};
  tile_split<P, V, U, S, EXT>(c, a.k, cs, tile * 64 * V * 4, part);
}
#endif

#if RAID6C_VARIANT >= 3
// Job-list kernels (variant 3: plans, plain code; variant 4: extended Q
// parity, k > p; variant 5: the server's small batches).  Work-groups of 4 waves; wave w of
// work-group b takes item 4b + w: a tile of 64 lanes x GV dwords of one job
// (any base, strip stride, row size, case), run by tile_recover_one_pass (one
// streaming pass for every case).  Jobs whose rows are not all on 128-byte lines load
// with the ordinary cache policy (the lines at tile edges are read by two
// waves); the others stream non-temporally.
// Vector width and strips per load batch, per prime: vec 2 (tiles of 512
// bytes) with four strips per batch up to p = 31; vec 2 with one strip per
// batch for 37..53 (alone on a 20,000-stripe mix, the p = 37 and 53 grids
// went from 67% to 72% of peak against vec 1 with four; two strips per batch
// measured the same); vec 1 with four above, where vec 2 spills.
// Variant 5 is for batches too small to fill the GPU, where a request's time
// is the time a wave takes to walk its tile through the strips: the S waves
// of a work-group share one tile and each walks a contiguous S-th of the
// strips, four at a time (tile_split, as the strided split-K kernels), with
// the widest tile whose S partials fit in 64 KiB of LDS: vec 2 with S = 4 up
// to p = 13, vec 1 with S = 4 up to p = 31, vec 1 with S = 2 above.
#if defined(RAID6C_GROUP_VEC)
constexpr int kGroupVec = RAID6C_GROUP_VEC;
#elif RAID6C_VARIANT == 5
constexpr int kGroupVec = kP <= 13 ? 2 : 1;
#else
constexpr int kGroupVec = kP <= 53 ? 2 : 1;
#endif
#if defined(RAID6C_GROUP_UNROLL)
constexpr int kGroupUnroll = RAID6C_GROUP_UNROLL;
#elif RAID6C_VARIANT == 5
constexpr int kGroupUnroll = 4;
#else
constexpr int kGroupUnroll = (kP > 31 && kP <= 53) ? 1 : 4;
#endif
#if RAID6C_VARIANT == 5
constexpr int kLatSplit = sk_lds_bytes_any(kGroupVec, 4) <= 65536 ? 4 : 2;
static_assert(sk_lds_bytes_any(kGroupVec, kLatSplit) <= 65536, "split partials exceed 64 KiB of LDS");
#endif
static_assert((kVecMask & kGroupVec) != 0, "job-list vector width not built");

// One column tile of one job, by one wave (EXT: extended Q parity).
template <int P, bool EXT>
__device__ __forceinline__ void group_item(const GroupArgs& a, uint32_t* smem) {
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t i = xcd_chunk(blockIdx.x, gridDim.x) * 4 + w;
  if (i >= a.nitems) return;
  const BatchItem item = a.items[i];
  const BatchJob& j = a.jobs[item.job];
  const uint32_t col = item.col + lane * (kGroupVec * 4);
  if (col >= j.row_bytes) return;
  const ColsJob c{j.base, j.strip_stride, j.out0, j.out1, j.src, j.src_stride, j.e0, j.e1,
                  j.row_bytes, col, (uint32_t)((P - 1) * j.row_bytes)};
  const Case cs{j.op, j.x, j.y};
  if (c.lines_aligned())
    tile_recover_one_pass<P, kGroupVec, kGroupUnroll, EXT>(c, j.k, cs, smem + threadIdx.x, 256);
  else
    tile_recover_one_pass<P, kGroupVec, kGroupUnroll, EXT>(c.with_policy<kLoadPolicyShared>(), j.k, cs,
                                                           smem + threadIdx.x, 256);
}

// Templates on P only so that profiles name each prime's grid.
#if RAID6C_VARIANT == 3
template <int P>
__global__ void __launch_bounds__(256) zp_group_kernel(const GroupArgs a) {
  extern __shared__ __align__(16) uint32_t smem[];
  group_item<P, false>(a, smem);
}
#elif RAID6C_VARIANT == 5
// One item per work-group of kLatSplit waves (plain code).
template <int P>
__global__ void __launch_bounds__(64 * kLatSplit) zp_group_lat_kernel(const GroupArgs a) {
  extern __shared__ __align__(16) uint32_t part[];
  const uint32_t i = xcd_chunk(blockIdx.x, gridDim.x);
  if (i >= a.nitems) return;   // uniform over the work-group
  const BatchItem item = a.items[i];
  const BatchJob& j = a.jobs[item.job];
  const uint32_t col = item.col + (threadIdx.x & 63) * (kGroupVec * 4);
  const ColsJob c{j.base, j.strip_stride, j.out0, j.out1, j.src, j.src_stride, j.e0, j.e1,
                  j.row_bytes, col, (uint32_t)((P - 1) * j.row_bytes)};
  const Case cs{j.op, j.x, j.y};
  if (c.lines_aligned())
    tile_split<P, kGroupVec, kGroupUnroll, kLatSplit, false>(c, j.k, cs, item.col, part);
  else
    tile_split<P, kGroupVec, kGroupUnroll, kLatSplit, false>(c.with_policy<kLoadPolicyShared>(), j.k, cs,
                                                            item.col, part);
}
#else
template <int P>
__global__ void __launch_bounds__(256) zp_group_ext_kernel(const GroupArgs a) {
  extern __shared__ __align__(16) uint32_t smem[];
  group_item<P, true>(a, smem);
}
#endif
#endif

// (vec, unroll) pairs built for this prime: accumulators take (2p-1)*vec
// dwords per thread and a batch of loads unroll*(p-1)*vec more.  Up to 400
// of the 512 VGPRs a wave can hold: for the large primes four strips per
// batch (one wave per SIMD) beat one (two or three waves) by 2-9%.
#ifndef RAID6C_REG_BUDGET
#define RAID6C_REG_BUDGET 400
#endif
template <int V, int U>
constexpr bool built() {
  return (kVecMask & V) != 0 && (2 * kP - 1) * V + U * (kP - 1) * V <= RAID6C_REG_BUDGET;
}

// Split factors S (2, 4) built with vector width V: the partials of S
// waves fit in 64 KiB of LDS.
constexpr int split_mask(int v) {
  return !(kVecMask & v) ? 0
                         : ((sk_lds_bytes_any(v, 2) <= 65536 ? 2 : 0) | (sk_lds_bytes_any(v, 4) <= 65536 ? 4 : 0));
}

constexpr int unroll_mask(int v) {
  return v == 1 ? ((built<1, 1>() ? 1 : 0) | (built<1, 2>() ? 2 : 0) | (built<1, 4>() ? 4 : 0))
       : v == 2 ? ((built<2, 1>() ? 1 : 0) | (built<2, 2>() ? 2 : 0) | (built<2, 4>() ? 4 : 0))
       : v == 4 ? ((built<4, 1>() ? 1 : 0) | (built<4, 2>() ? 2 : 0) | (built<4, 4>() ? 4 : 0))
                : 0;
}

template <int V, int U, int LP>
hipError_t launch_lp(ZpKind kind, const ZpConfig& cfg, const ZpArgs& a, uint32_t grid,
                     hipStream_t stream) {
  if constexpr (built<V, U>() && RAID6C_VARIANT < 3) {
#if RAID6C_VARIANT == 2
    (void)kind;
    const dim3 g(grid);
    const bool ext = a.k > kP;
    if constexpr ((split_mask(V) & 2) != 0) {
      if (cfg.split == 2) {
        if (ext) hipLaunchKernelGGL((zp_split_kernel<kP, V, U, 2, true, LP>), g, dim3(128), sk_lds_bytes_any(V, 2), stream, a);
        else hipLaunchKernelGGL((zp_split_kernel<kP, V, U, 2, false, LP>), g, dim3(128), sk_lds_bytes_any(V, 2), stream, a);
        return hipGetLastError();
      }
    }
    if constexpr ((split_mask(V) & 4) != 0) {
      if (cfg.split == 4) {
        if (ext) hipLaunchKernelGGL((zp_split_kernel<kP, V, U, 4, true, LP>), g, dim3(256), sk_lds_bytes_any(V, 4), stream, a);
        else hipLaunchKernelGGL((zp_split_kernel<kP, V, U, 4, false, LP>), g, dim3(256), sk_lds_bytes_any(V, 4), stream, a);
        return hipGetLastError();
      }
    }
    return hipErrorInvalidValue;
#else
    if ((a.k > kP) != kExt) return hipErrorInvalidValue;
    const dim3 g(grid), b(cfg.threads);
    const size_t lds = (size_t)kP * cfg.threads * 4;
    if (kind == KIND_ENCODE) hipLaunchKernelGGL((zp_encode_kernel<kP, V, U, kExt, LP>), g, b, 0, stream, a);
    else hipLaunchKernelGGL((zp_recover_kernel<kP, V, U, kExt, LP>), g, b, lds, stream, a);
    return hipGetLastError();
#endif
  } else {
    return hipErrorInvalidValue;
  }
}

template <int V, int U>
hipError_t launch_vu(ZpKind kind, const ZpConfig& cfg, const ZpArgs& a, uint32_t grid,
                     hipStream_t stream) {
  if (a.shared_lines) return launch_lp<V, U, kLoadPolicyShared>(kind, cfg, a, grid, stream);
  return launch_lp<V, U, RAID6C_LOAD_POLICY>(kind, cfg, a, grid, stream);
}

hipError_t launch_here(ZpKind kind, const ZpConfig& cfg, const ZpArgs& a, uint32_t grid,
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

// Launchers of the other objects of this prime.
hipError_t RAID6C_CAT(zp_launch_ext_, RAID6C_P)(ZpKind kind, const ZpConfig& cfg, const ZpArgs& a, uint32_t grid,
                                                hipStream_t stream);
hipError_t RAID6C_CAT(zp_launch_split_, RAID6C_P)(ZpKind kind, const ZpConfig& cfg, const ZpArgs& a, uint32_t grid,
                                                  hipStream_t stream);
void RAID6C_CAT(zp_group_shape_, RAID6C_P)(ZpPrimeEntry& e);
void RAID6C_CAT(zp_group_ext_shape_, RAID6C_P)(ZpPrimeEntry& e);
void RAID6C_CAT(zp_group_lat_shape_, RAID6C_P)(ZpPrimeEntry& e);

#if RAID6C_VARIANT == 3
void RAID6C_CAT(zp_group_shape_, RAID6C_P)(ZpPrimeEntry& e) {
  e.group_kernel = (const void*)zp_group_kernel<kP>;
  e.group_vec = kGroupVec;
  e.group_per_wg = 4;
  e.group_threads = 256;
  e.group_lds = kP * 256 * 4;
}
#elif RAID6C_VARIANT == 5
// One item per work-group of kLatSplit waves; its own tile width.
void RAID6C_CAT(zp_group_lat_shape_, RAID6C_P)(ZpPrimeEntry& e) {
  e.group_lat_kernel = (const void*)zp_group_lat_kernel<kP>;
  e.group_lat_vec = kGroupVec;
  e.group_lat_threads = 64 * kLatSplit;
  e.group_lat_lds = sk_lds_bytes_any(kGroupVec, kLatSplit);
}
#elif RAID6C_VARIANT == 4
// Same tiles and launch shape as the plain job-list kernel (same constants).
void RAID6C_CAT(zp_group_ext_shape_, RAID6C_P)(ZpPrimeEntry& e) {
  e.group_ext_kernel = (const void*)zp_group_ext_kernel<kP>;
  e.group_ext_vec = kGroupVec;
}
#elif RAID6C_VARIANT == 1
hipError_t RAID6C_CAT(zp_launch_ext_, RAID6C_P)(ZpKind kind, const ZpConfig& cfg, const ZpArgs& a, uint32_t grid,
                                                hipStream_t stream) {
  return launch_here(kind, cfg, a, grid, stream);
}
#elif RAID6C_VARIANT == 2
hipError_t RAID6C_CAT(zp_launch_split_, RAID6C_P)(ZpKind kind, const ZpConfig& cfg, const ZpArgs& a, uint32_t grid,
                                                  hipStream_t stream) {
  return launch_here(kind, cfg, a, grid, stream);
}
#else
namespace {
// Plain code; split-K configurations (plain or extended) go to the split object.
hipError_t launch_plain(ZpKind kind, const ZpConfig& cfg, const ZpArgs& a, uint32_t grid, hipStream_t stream) {
  if (cfg.split > 1) return RAID6C_CAT(zp_launch_split_, RAID6C_P)(kind, cfg, a, grid, stream);
  return launch_here(kind, cfg, a, grid, stream);
}

ZpPrimeEntry make_entry() {
  ZpPrimeEntry e{kP, &launch_plain, &RAID6C_CAT(zp_launch_ext_, RAID6C_P), kVecMask,
                 {0, unroll_mask(1), unroll_mask(2), 0, unroll_mask(4)},
                 {0, split_mask(1), split_mask(2), 0, split_mask(4)},
                 nullptr, 0, 0, 0, 0, nullptr, 0, nullptr, 0, 0, 0};
  RAID6C_CAT(zp_group_shape_, RAID6C_P)(e);
  RAID6C_CAT(zp_group_ext_shape_, RAID6C_P)(e);
  RAID6C_CAT(zp_group_lat_shape_, RAID6C_P)(e);
  return e;
}
}  // namespace

const ZpPrimeEntry* RAID6C_CAT(zp_entry_, RAID6C_P)() {
  static const ZpPrimeEntry e = make_entry();
  return &e;
}
#endif

}  // namespace raid6c
