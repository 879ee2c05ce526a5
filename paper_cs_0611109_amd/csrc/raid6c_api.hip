// raid6c_api.hip -- the C ABI of libraid6c (declared in include/raid6c.h):
// argument checks, launch configuration and kernel launches.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/raid6c.h"
#include "raid6c_internal.h"
#include "tune.h"

namespace raid6c {

#define RAID6C_PRIMES(X) \
  X(3) X(5) X(7) X(11) X(13) X(17) X(19) X(23) X(29) X(31) X(37) X(41) X(43) X(47) X(53) X(59) X(61)

#define RAID6C_DECL(p) const ZpPrimeEntry* zp_entry_##p();
RAID6C_PRIMES(RAID6C_DECL)
#undef RAID6C_DECL

const ZpPrimeEntry* zp_prime_entry(int p) {
  switch (p) {
#define RAID6C_CASE(q) \
  case q:              \
    return zp_entry_##q();
    RAID6C_PRIMES(RAID6C_CASE)
#undef RAID6C_CASE
    default:
      return nullptr;
  }
}

static thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

static bool is_odd_prime(int p) {
  if (p < 3 || (p % 2) == 0) return false;
  for (int d = 3; d * d <= p; d += 2)
    if (p % d == 0) return false;
  return true;
}

static bool aligned16(const void* ptr) { return ((uintptr_t)ptr & 15u) == 0; }

// F2[X] polynomials of degree < 64 as bit masks (bit i = coefficient of X^i).
static int poly_deg(uint64_t a) { return 63 - __builtin_clzll(a); }

static uint64_t poly_rem(uint64_t a, uint64_t m) {
  const int dm = poly_deg(m);
  while (a != 0 && poly_deg(a) >= dm) a ^= m << (poly_deg(a) - dm);
  return a;
}

static uint64_t poly_gcd(uint64_t a, uint64_t b) {
  while (b != 0) {
    const uint64_t r = poly_rem(a, b);
    a = b;
    b = r;
  }
  return a;
}

// Theorem 3.3.3, condition (3): for every 0 < m < p, X^p + 1 and X^m + X + 1
// are relatively prime over F2.  Exactly then the 2p-1 elements x^i and
// 1 + x^j form a cone and the extended Q parity protects 2p-1 data strips.
// (p <= kMaxPrime = 61, so X^p + 1 fits in 64 bits.)
static bool extension_ok(int p) {
  const uint64_t xp1 = (1ull << p) | 1ull;
  for (int m = 1; m < p; ++m)
    if (poly_gcd(xp1, (1ull << m) ^ 2ull ^ 1ull) != 1ull) return false;
  return true;
}

// Largest k for a supported prime: 2p-1 with the extended Q parity, else p.
static int max_data(int p) {
  static const auto table = [] {
    struct T { int k[kMaxPrime + 1]; } t{};
    for (int q = 3; q <= kMaxPrime; q += 2)
      if (is_odd_prime(q)) t.k[q] = extension_ok(q) ? 2 * q - 1 : q;
    return t;
  }();
  return table.k[p];
}

// Common checks of p, k and the row size.
int check_geometry(int p, int k, size_t row_bytes) {
  if (!is_odd_prime(p)) return fail(RAID6C_E_ARG, "p = %d is not an odd prime", p);
  if (p > kMaxPrime)
    return fail(RAID6C_E_UNSUPPORTED, "p = %d exceeds the largest built prime %d", p, kMaxPrime);
  if (k < 1 || k > max_data(p))
    return fail(RAID6C_E_ARG, "k = %d must satisfy 1 <= k <= %d for p = %d%s", k, max_data(p), p,
                max_data(p) == p ? " (p fails Theorem 3.3.3: no extended Q parity)" : "");
  if (row_bytes == 0 || (row_bytes % 16) != 0)
    return fail(RAID6C_E_ARG, "row_bytes = %zu must be a positive multiple of 16", row_bytes);
  if ((size_t)(p - 1) * row_bytes >= ((size_t)1 << 31))
    return fail(RAID6C_E_ARG, "a strip of (p-1)*row_bytes = %zu bytes must stay below 2 GiB",
                (size_t)(p - 1) * row_bytes);
  return RAID6C_OK;
}

static int check_strided(int p, int k, size_t row_bytes, const void* base, size_t strip_stride,
                         size_t stripe_stride, size_t nstripes) {
  int rc = check_geometry(p, k, row_bytes);
  if (rc != RAID6C_OK) return rc;
  if (nstripes == 0) return RAID6C_OK;
  if (base == nullptr || !aligned16(base)) return fail(RAID6C_E_ARG, "base is NULL or not 16-byte aligned");
  const size_t strip = (size_t)(p - 1) * row_bytes;
  if ((strip_stride % 16) != 0 || strip_stride < strip)
    return fail(RAID6C_E_ARG, "strip_stride = %zu must be a multiple of 16 and >= (p-1)*row_bytes = %zu",
                strip_stride, strip);
  if (nstripes > 1 && ((stripe_stride % 16) != 0 || stripe_stride < (size_t)(k + 2) * strip_stride))
    return fail(RAID6C_E_ARG,
                "stripe_stride = %zu must be a multiple of 16 and >= (k+2)*strip_stride = %zu",
                stripe_stride, (size_t)(k + 2) * strip_stride);
  if (nstripes > 0xFFFFFFFFull) return fail(RAID6C_E_ARG, "nstripes exceeds 2^32-1");
  return RAID6C_OK;
}

static int check_strip_ptrs(int n, const void* const* ptrs, size_t strip_bytes) {
  if (ptrs == nullptr) return fail(RAID6C_E_ARG, "strip pointer array is NULL");
  for (int j = 0; j < n; ++j) {
    if (ptrs[j] == nullptr || !aligned16(ptrs[j]))
      return fail(RAID6C_E_ARG, "strip %d is NULL or not 16-byte aligned", j);
  }
  for (int i = 0; i < n; ++i) {
    const uintptr_t a0 = (uintptr_t)ptrs[i];
    for (int j = i + 1; j < n; ++j) {
      const uintptr_t b0 = (uintptr_t)ptrs[j];
      if (a0 < b0 + strip_bytes && b0 < a0 + strip_bytes)
        return fail(RAID6C_E_ARG, "strips %d and %d overlap", i, j);
    }
  }
  return RAID6C_OK;
}

// Multiplier of work-group order 2: near n / golden ratio, coprime with n,
// so that s -> m*s mod n permutes the n stripes of a launch and places
// consecutive work-groups far apart.
static uint32_t scatter_multiplier(size_t n) {
  if (n < 3) return 1u;
  uint64_t m = (uint64_t)((double)n * 0.6180339887498949);
  if (m < 1) m = 1;
  auto gcd = [](uint64_t a, uint64_t b) {
    while (b != 0) {
      const uint64_t t = a % b;
      a = b;
      b = t;
    }
    return a;
  };
  while (gcd(m, n) != 1) ++m;
  return (uint32_t)m;
}

// Launch a Z_p kernel over `nstripes` stripes, splitting the grid when needed.
static int launch_zp(int p, ZpKind kind, ZpArgs a, size_t nstripes, void* stream) {
  if (nstripes == 0) return RAID6C_OK;
  const ZpPrimeEntry* e = zp_prime_entry(p);
  if (e == nullptr) return fail(RAID6C_E_UNSUPPORTED, "p = %d is not built", p);
  const ZpConfig cfg = choose_config(*e, tune_slot(kind, a.k > p), a.row_bytes);
  // A split-K work-group covers 64 lanes x vec dwords of a row;
  // otherwise every thread its own vec dwords.
  const bool split = cfg.split > 1;
  const uint64_t tile_bytes = (uint64_t)(split ? 64 : cfg.threads) * cfg.vec * 4;
  a.tiles = (uint32_t)((a.row_bytes + tile_bytes - 1) / tile_bytes);
  // Rows that do not all start on 128-byte lines are loaded with the
  // ordinary cache policy (the kernels' LP parameter).
  uint64_t addr_bits = a.stripe_stride | a.row_bytes | (uintptr_t)a.src_base | a.src_strip_stride |
                       a.src_stripe_stride;
  for (int j = 0; j < a.k + 2; ++j) addr_bits |= (uintptr_t)a.strip[j];
  a.shared_lines = (addr_bits & 127u) != 0;
  a.xcd_order = cfg.order == 1 || (a.shared_lines && cfg.order == 0);
  // Keep grid * threads below 2^31.
  const uint64_t max_blocks = (((uint64_t)1 << 31) / cfg.threads);
  const uint64_t chunk = max_blocks / a.tiles;
  size_t done = 0;
  while (done < nstripes) {
    const size_t n = (nstripes - done) < chunk ? (nstripes - done) : chunk;
    ZpArgs b = a;
    b.kind = kind;
    if (done != 0) {
      for (int j = 0; j < a.k + 2; ++j) b.strip[j] = a.strip[j] + done * a.stripe_stride;
      if (a.erasures != nullptr) b.erasures = a.erasures + 2 * done;
      if (a.src_base != nullptr) b.src_base = a.src_base + done * a.src_stripe_stride;
    }
    b.nstripes = (uint32_t)n;
    b.stripe_mult = cfg.order == 2 ? scatter_multiplier(n) : 0u;
    // Split-K configurations (plain or extended) go through the plain entry,
    // which hands them to the split object.
    const ZpLauncher fn = (a.k > p && !split) ? e->launch_ext : e->launch;
    const hipError_t err = fn(kind, cfg, b, (uint32_t)(n * a.tiles), (hipStream_t)stream);
    if (err != hipSuccess) return fail(RAID6C_E_HIP, "kernel launch failed: %s", hipGetErrorString(err));
    done += n;
  }
  return RAID6C_OK;
}

static ZpArgs strided_args(int k, size_t row_bytes, void* base, size_t strip_stride, size_t stripe_stride) {
  ZpArgs a;
  memset(&a, 0, sizeof a);
  for (int j = 0; j < k + 2; ++j) a.strip[j] = (uint8_t*)base + (size_t)j * strip_stride;
  a.stripe_stride = stripe_stride;
  a.row_bytes = row_bytes;
  a.k = k;
  a.e0 = -1;
  a.e1 = -1;
  return a;
}

}  // namespace raid6c

using namespace raid6c;

extern "C" {

int raid6c_max_prime(void) { return kMaxPrime; }

int raid6c_is_supported_prime(int p) { return (is_odd_prime(p) && p <= kMaxPrime) ? 1 : 0; }

int raid6c_max_data_strips(int p) {
  g_last_error.clear();
  if (!is_odd_prime(p)) return fail(RAID6C_E_ARG, "p = %d is not an odd prime", p);
  if (p > kMaxPrime) return fail(RAID6C_E_UNSUPPORTED, "p = %d exceeds the largest built prime %d", p, kMaxPrime);
  return max_data(p);
}

const char* raid6c_strerror(int code) {
  switch (code) {
    case RAID6C_OK: return "success";
    case RAID6C_E_ARG: return "invalid argument";
    case RAID6C_E_UNSUPPORTED: return "unsupported by the GPU path";
    case RAID6C_E_HIP: return "HIP runtime error";
    case RAID6C_E_NOMEM: return "out of memory";
    case RAID6C_E_STATE: return "invalid state";
    default: return "unknown error";
  }
}

const char* raid6c_last_error(void) { return g_last_error.c_str(); }

int raid6c_encode(int p, int k, size_t row_bytes, const void* const* data, void* P, void* Q, void* stream) {
  g_last_error.clear();
  int rc = check_geometry(p, k, row_bytes);
  if (rc != RAID6C_OK) return rc;
  if (data == nullptr) return fail(RAID6C_E_ARG, "data pointer array is NULL");
  const void* ptrs[kMaxStrips];
  for (int j = 0; j < k; ++j) ptrs[j] = data[j];
  ptrs[k] = P;
  ptrs[k + 1] = Q;
  rc = check_strip_ptrs(k + 2, ptrs, (size_t)(p - 1) * row_bytes);
  if (rc != RAID6C_OK) return rc;
  ZpArgs a;
  memset(&a, 0, sizeof a);
  for (int j = 0; j < k + 2; ++j) a.strip[j] = (uint8_t*)ptrs[j];
  a.row_bytes = row_bytes;
  a.k = k;
  a.e0 = a.e1 = -1;
  return launch_zp(p, KIND_ENCODE, a, 1, stream);
}

static int recover_single_stripe(int p, int k, size_t row_bytes, void* const* strips, int e0, int e1,
                                 void* stream) {
  g_last_error.clear();
  int rc = check_geometry(p, k, row_bytes);
  if (rc != RAID6C_OK) return rc;
  if (classify(k, e0, e1).op == OP_BAD)
    return fail(RAID6C_E_ARG, "invalid erasures (%d, %d) for k = %d", e0, e1, k);
  rc = check_strip_ptrs(k + 2, (const void* const*)strips, (size_t)(p - 1) * row_bytes);
  if (rc != RAID6C_OK) return rc;
  ZpArgs a;
  memset(&a, 0, sizeof a);
  for (int j = 0; j < k + 2; ++j) a.strip[j] = (uint8_t*)strips[j];
  a.row_bytes = row_bytes;
  a.k = k;
  a.e0 = e0;
  a.e1 = e1;
  return launch_zp(p, KIND_RECOVER, a, 1, stream);
}

int raid6c_recover_1(int p, int k, size_t row_bytes, void* const* strips, int e, void* stream) {
  if (e < 0 || e > k + 1) {
    g_last_error.clear();
    return fail(RAID6C_E_ARG, "erased strip %d out of range 0..%d", e, k + 1);
  }
  return recover_single_stripe(p, k, row_bytes, strips, e, -1, stream);
}

int raid6c_recover_2(int p, int k, size_t row_bytes, void* const* strips, int e0, int e1, void* stream) {
  if (e0 < 0 || e1 < 0 || e0 > k + 1 || e1 > k + 1 || e0 == e1) {
    g_last_error.clear();
    return fail(RAID6C_E_ARG, "erased strips (%d, %d) must be distinct and in 0..%d", e0, e1, k + 1);
  }
  return recover_single_stripe(p, k, row_bytes, strips, e0, e1, stream);
}

int raid6c_write(int p, int k, size_t row_bytes, const void* src, size_t src_strip_stride, void* const* strips,
                 void* stream) {
  g_last_error.clear();
  int rc = check_geometry(p, k, row_bytes);
  if (rc != RAID6C_OK) return rc;
  const size_t strip = (size_t)(p - 1) * row_bytes;
  if (src == nullptr || !aligned16(src)) return fail(RAID6C_E_ARG, "src is NULL or not 16-byte aligned");
  if ((src_strip_stride % 16) != 0 || src_strip_stride < strip)
    return fail(RAID6C_E_ARG, "src_strip_stride must be a multiple of 16 and >= (p-1)*row_bytes");
  rc = check_strip_ptrs(k + 2, (const void* const*)strips, strip);
  if (rc != RAID6C_OK) return rc;
  const uintptr_t s0 = (uintptr_t)src, s1 = s0 + (uintptr_t)(k - 1) * src_strip_stride + strip;
  for (int j = 0; j < k + 2; ++j) {
    const uintptr_t a0 = (uintptr_t)strips[j];
    if (a0 < s1 && s0 < a0 + strip) return fail(RAID6C_E_ARG, "the payload overlaps strip %d", j);
  }
  ZpArgs a;
  memset(&a, 0, sizeof a);
  for (int j = 0; j < k + 2; ++j) a.strip[j] = (uint8_t*)strips[j];
  a.row_bytes = row_bytes;
  a.k = k;
  a.e0 = a.e1 = -1;
  a.src_base = (const uint8_t*)src;
  a.src_strip_stride = src_strip_stride;
  return launch_zp(p, KIND_ENCODE, a, 1, stream);
}

int raid6c_read_degraded(int p, int k, size_t row_bytes, const void* const* strips, int e0, int e1, void* out,
                         void* stream) {
  g_last_error.clear();
  int rc = check_geometry(p, k, row_bytes);
  if (rc != RAID6C_OK) return rc;
  if (strips == nullptr) return fail(RAID6C_E_ARG, "strip pointer array is NULL");
  if (e0 < 0 || e0 > k + 1 || e1 < -1 || e1 > k + 1 || e0 == e1)
    return fail(RAID6C_E_ARG, "erased strips (%d, %d) must be distinct and in 0..%d", e0, e1, k + 1);
  if (out == nullptr || !aligned16(out)) return fail(RAID6C_E_ARG, "out is NULL or not 16-byte aligned");
  const size_t strip = (size_t)(p - 1) * row_bytes;
  const int lo = (e1 < 0 || e0 < e1) ? e0 : e1;
  const int hi = (e1 < 0) ? -1 : (e0 < e1 ? e1 : e0);
  const void* table[kMaxStrips];
  for (int j = 0; j < k + 2; ++j) table[j] = strips[j];
  table[lo] = out;
  if (hi >= 0) table[hi] = (uint8_t*)out + strip;
  rc = check_strip_ptrs(k + 2, table, strip);
  if (rc != RAID6C_OK) return rc;
  ZpArgs a;
  memset(&a, 0, sizeof a);
  for (int j = 0; j < k + 2; ++j) a.strip[j] = (uint8_t*)table[j];
  a.row_bytes = row_bytes;
  a.k = k;
  a.e0 = e0;
  a.e1 = e1;
  return launch_zp(p, KIND_RECOVER, a, 1, stream);
}

int raid6c_encode_n(int p, int k, size_t row_bytes, void* base, size_t strip_stride, size_t stripe_stride,
                    size_t nstripes, void* stream) {
  g_last_error.clear();
  int rc = check_strided(p, k, row_bytes, base, strip_stride, stripe_stride, nstripes);
  if (rc != RAID6C_OK || nstripes == 0) return rc;
  ZpArgs a = strided_args(k, row_bytes, base, strip_stride, stripe_stride);
  return launch_zp(p, KIND_ENCODE, a, nstripes, stream);
}

int raid6c_recover_n(int p, int k, size_t row_bytes, void* base, size_t strip_stride, size_t stripe_stride,
                     size_t nstripes, const int32_t* erasures, int32_t* bad_count, void* stream) {
  g_last_error.clear();
  int rc = check_strided(p, k, row_bytes, base, strip_stride, stripe_stride, nstripes);
  if (rc != RAID6C_OK) return rc;
  if (nstripes == 0) return RAID6C_OK;
  if (erasures == nullptr || ((uintptr_t)erasures & 3u) != 0)
    return fail(RAID6C_E_ARG, "erasures is NULL or not 4-byte aligned");
  if (bad_count != nullptr && ((uintptr_t)bad_count & 3u) != 0)
    return fail(RAID6C_E_ARG, "bad_count is not 4-byte aligned");
  ZpArgs a = strided_args(k, row_bytes, base, strip_stride, stripe_stride);
  a.erasures = erasures;
  a.bad_count = bad_count;
  return launch_zp(p, KIND_RECOVER, a, nstripes, stream);
}

static int rs_run(int k, size_t strip_bytes, void* base, size_t strip_stride, size_t stripe_stride,
                  size_t nstripes, const int32_t* erasures, int32_t* bad_count, void* stream) {
  g_last_error.clear();
  if (k < 1 || k > 255) return fail(RAID6C_E_ARG, "k = %d must satisfy 1 <= k <= 255", k);
  if (strip_bytes == 0 || (strip_bytes % 16) != 0 || strip_bytes >= ((size_t)1 << 31))
    return fail(RAID6C_E_ARG, "strip_bytes = %zu must be a positive multiple of 16 below 2 GiB", strip_bytes);
  if (nstripes == 0) return RAID6C_OK;
  if (base == nullptr || !aligned16(base)) return fail(RAID6C_E_ARG, "base is NULL or not 16-byte aligned");
  if ((strip_stride % 16) != 0 || strip_stride < strip_bytes)
    return fail(RAID6C_E_ARG, "strip_stride must be a multiple of 16 and >= strip_bytes");
  if (nstripes > 1 && ((stripe_stride % 16) != 0 || stripe_stride < (size_t)(k + 2) * strip_stride))
    return fail(RAID6C_E_ARG, "stripe_stride must be a multiple of 16 and >= (k+2)*strip_stride");
  if (nstripes > 0xFFFFFFFFull) return fail(RAID6C_E_ARG, "nstripes exceeds 2^32-1");
  if (erasures != nullptr && ((uintptr_t)erasures & 3u) != 0)
    return fail(RAID6C_E_ARG, "erasures must be 4-byte aligned");
  const RsConfig cfg = choose_rs_config(strip_bytes, erasures != nullptr);
  RsArgs a;
  memset(&a, 0, sizeof a);
  a.strip_stride = strip_stride;
  a.stripe_stride = stripe_stride;
  a.strip_bytes = strip_bytes;
  a.k = k;
  a.bad_count = bad_count;
  const uint64_t tile_bytes = (uint64_t)cfg.threads * cfg.vec * 4;
  a.tiles = (uint32_t)((strip_bytes + tile_bytes - 1) / tile_bytes);
  const uint64_t chunk = (((uint64_t)1 << 31) / cfg.threads) / a.tiles;
  size_t done = 0;
  while (done < nstripes) {
    const size_t n = (nstripes - done) < chunk ? (nstripes - done) : chunk;
    a.base = (uint8_t*)base + done * stripe_stride;
    a.erasures = erasures != nullptr ? erasures + 2 * done : nullptr;
    a.nstripes = (uint32_t)n;
    const hipError_t err =
        rs_launch(a, cfg.vec, cfg.unroll, cfg.threads, (uint32_t)(n * a.tiles), (hipStream_t)stream);
    if (err != hipSuccess) return fail(RAID6C_E_HIP, "kernel launch failed: %s", hipGetErrorString(err));
    done += n;
  }
  return RAID6C_OK;
}

int raid6c_rs_encode_n(int k, size_t strip_bytes, void* base, size_t strip_stride, size_t stripe_stride,
                       size_t nstripes, void* stream) {
  return rs_run(k, strip_bytes, base, strip_stride, stripe_stride, nstripes, nullptr, nullptr, stream);
}

// Small writes (update.hip): launch over nstripes stripes, splitting the grid.
static int launch_update(int p, UpdArgs a, size_t nstripes, void* stream) {
  if (nstripes == 0) return RAID6C_OK;
  const int vec = (p <= 13 && a.row_bytes >= 512) ? 2 : 1;
#ifndef RAID6C_UPDATE_THREADS
#define RAID6C_UPDATE_THREADS 128
#endif
  int threads = 64;
  while (threads < RAID6C_UPDATE_THREADS && (uint64_t)threads * vec * 4 < a.row_bytes) threads *= 2;
  const uint64_t tile_bytes = (uint64_t)threads * vec * 4;
  a.tiles = (uint32_t)((a.row_bytes + tile_bytes - 1) / tile_bytes);
  const uint64_t addr_bits = a.row_bytes | (uintptr_t)a.base | a.strip_stride | a.stripe_stride |
                             (uintptr_t)a.src | a.src_stride | (uintptr_t)a.pd | (uintptr_t)a.pp | (uintptr_t)a.pq;
  const bool shared_lines = (addr_bits & 127u) != 0;
  const uint64_t chunk = (((uint64_t)1 << 31) / threads) / a.tiles;
  size_t done = 0;
  while (done < nstripes) {
    const size_t n = (nstripes - done) < chunk ? (nstripes - done) : chunk;
    UpdArgs b = a;
    if (done != 0) {
      b.base = a.base + done * a.stripe_stride;
      b.src = a.src + done * a.src_stride;
      if (a.targets != nullptr) b.targets = a.targets + done;
    }
    b.nstripes = (uint32_t)n;
    const hipError_t err =
        update_launch(b, p, vec, threads, (uint32_t)(n * a.tiles), shared_lines, (hipStream_t)stream);
    if (err != hipSuccess) return fail(RAID6C_E_HIP, "kernel launch failed: %s", hipGetErrorString(err));
    done += n;
  }
  return RAID6C_OK;
}

int raid6c_update(int p, int k, size_t row_bytes, void* const* strips, int t, const void* new_strip, void* stream) {
  g_last_error.clear();
  int rc = check_geometry(p, k, row_bytes);
  if (rc != RAID6C_OK) return rc;
  if (t < 0 || t >= k) return fail(RAID6C_E_ARG, "t = %d must index a data strip (0..%d)", t, k - 1);
  if (strips == nullptr) return fail(RAID6C_E_ARG, "strip pointer array is NULL");
  const size_t strip = (size_t)(p - 1) * row_bytes;
  const void* ptrs[4] = {strips[t], strips[k], strips[k + 1], new_strip};
  rc = check_strip_ptrs(4, ptrs, strip);
  if (rc != RAID6C_OK) return rc;
  UpdArgs a;
  memset(&a, 0, sizeof a);
  a.pd = (uint8_t*)strips[t];
  a.pp = (uint8_t*)strips[k];
  a.pq = (uint8_t*)strips[k + 1];
  a.src = (const uint8_t*)new_strip;
  a.row_bytes = row_bytes;
  a.t = t;
  a.k = k;
  return launch_update(p, a, 1, stream);
}

int raid6c_update_n(int p, int k, size_t row_bytes, void* base, size_t strip_stride, size_t stripe_stride,
                    size_t nstripes, const int32_t* targets, const void* src, size_t src_stride, int32_t* bad_count,
                    void* stream) {
  g_last_error.clear();
  int rc = check_strided(p, k, row_bytes, base, strip_stride, stripe_stride, nstripes);
  if (rc != RAID6C_OK) return rc;
  if (nstripes == 0) return RAID6C_OK;
  if (targets == nullptr || ((uintptr_t)targets & 3u) != 0)
    return fail(RAID6C_E_ARG, "targets is NULL or not 4-byte aligned");
  const size_t strip = (size_t)(p - 1) * row_bytes;
  if (src == nullptr || !aligned16(src)) return fail(RAID6C_E_ARG, "src is NULL or not 16-byte aligned");
  if (nstripes > 1 && ((src_stride % 16) != 0 || src_stride < strip))
    return fail(RAID6C_E_ARG, "src_stride = %zu must be a multiple of 16 and >= (p-1)*row_bytes = %zu", src_stride,
                strip);
  UpdArgs a;
  memset(&a, 0, sizeof a);
  a.base = (uint8_t*)base;
  a.strip_stride = strip_stride;
  a.stripe_stride = stripe_stride;
  a.src = (const uint8_t*)src;
  a.src_stride = src_stride;
  a.targets = targets;
  a.bad_count = bad_count;
  a.row_bytes = row_bytes;
  a.t = -1;
  a.k = k;
  return launch_update(p, a, nstripes, stream);
}

static int z17_convert(bool to_vertical, const void* in, size_t row_bytes, size_t count, void* out, void* stream) {
  g_last_error.clear();
  if (row_bytes == 0 || (row_bytes % 16) != 0)
    return fail(RAID6C_E_ARG, "row_bytes = %zu must be a positive multiple of 16", row_bytes);
  if (count == 0) return RAID6C_OK;
  if (in == nullptr || out == nullptr || !aligned16(in) || !aligned16(out))
    return fail(RAID6C_E_ARG, "a buffer is NULL or not 16-byte aligned");
  const size_t bytes = 16 * row_bytes;           // per strip, in either layout
  if (count > ((size_t)1 << 40) / bytes) return fail(RAID6C_E_ARG, "count * 16 * row_bytes is too large");
  const uintptr_t a0 = (uintptr_t)in, b0 = (uintptr_t)out;
  if (a0 < b0 + count * bytes && b0 < a0 + count * bytes)
    return fail(RAID6C_E_ARG, "input and output overlap");
  const hipError_t err = z17_launch(to_vertical, in, out, row_bytes, count, (hipStream_t)stream);
  if (err != hipSuccess) return fail(RAID6C_E_HIP, "kernel launch failed: %s", hipGetErrorString(err));
  return RAID6C_OK;
}

int raid6c_z17_to_vertical(const void* words, size_t row_bytes, size_t count, void* strips, void* stream) {
  return z17_convert(true, words, row_bytes, count, strips, stream);
}

int raid6c_z17_to_horizontal(const void* strips, size_t row_bytes, size_t count, void* words, void* stream) {
  return z17_convert(false, strips, row_bytes, count, words, stream);
}

int raid6c_rs_set_config(int vec, int unroll, int threads) {
  g_last_error.clear();
  if (!set_rs_override(vec, unroll, threads))
    return fail(RAID6C_E_ARG, "RS configuration (vec %d, unroll %d, threads %d) is not built", vec, unroll, threads);
  return RAID6C_OK;
}

int raid6c_rs_recover_n(int k, size_t strip_bytes, void* base, size_t strip_stride, size_t stripe_stride,
                        size_t nstripes, const int32_t* erasures, int32_t* bad_count, void* stream) {
  if (nstripes != 0 && erasures == nullptr) {
    g_last_error.clear();
    return fail(RAID6C_E_ARG, "erasures is NULL");
  }
  return rs_run(k, strip_bytes, base, strip_stride, stripe_stride, nstripes, erasures, bad_count, stream);
}

int raid6c_vec_mask(int p) {
  const ZpPrimeEntry* e = zp_prime_entry(p);
  return e ? e->vec_mask : 0;
}

int raid6c_unroll_mask(int p, int vec) {
  const ZpPrimeEntry* e = zp_prime_entry(p);
  if (e == nullptr || !(vec == 1 || vec == 2 || vec == 4)) return 0;
  return e->unroll_mask[vec];
}

int raid6c_tune_set(int p, int op, size_t row_bytes, int vec, int unroll, int threads, int split, int order) {
  g_last_error.clear();
  const ZpPrimeEntry* e = zp_prime_entry(p);
  if (e == nullptr) return fail(RAID6C_E_ARG, "p = %d is not built", p);
  if (op < 0 || op > 3)
    return fail(RAID6C_E_ARG, "op = %d must be 0 (encode), 1 (recovery), 2 or 3 (the same, k > p)", op);
  if (!e->has(vec, unroll))
    return fail(RAID6C_E_ARG, "(vec = %d, unroll = %d) is not built for p = %d", vec, unroll, p);
  if (!(threads == 64 || threads == 128 || threads == 256))
    return fail(RAID6C_E_ARG, "threads = %d must be 64, 128 or 256", threads);
  if (!e->has(ZpConfig{vec, unroll, threads, split}))
    return fail(RAID6C_E_ARG, "split = %d is not built for p = %d, vec = %d with threads = %d", split, p, vec,
                threads);
  if (order < 0 || order > 2) return fail(RAID6C_E_ARG, "order = %d must be 0, 1 or 2", order);
  if (row_bytes == 0) return fail(RAID6C_E_ARG, "row_bytes must be positive");
  set_tuned(p, op, row_bucket(row_bytes), ZpConfig{vec, unroll, threads, split, order});
  return RAID6C_OK;
}

int raid6c_tune_get(int p, int op, size_t row_bytes, int* vec, int* unroll, int* threads, int* split,
                    int* order) {
  g_last_error.clear();
  const ZpPrimeEntry* e = zp_prime_entry(p);
  if (e == nullptr) return fail(RAID6C_E_ARG, "p = %d is not built", p);
  if (op < 0 || op > 3)
    return fail(RAID6C_E_ARG, "op = %d must be 0 (encode), 1 (recovery), 2 or 3 (the same, k > p)", op);
  if (vec == nullptr || unroll == nullptr || threads == nullptr || split == nullptr || order == nullptr)
    return fail(RAID6C_E_ARG, "NULL output");
  const ZpConfig c = choose_config(*e, op, row_bytes);
  *vec = c.vec;
  *unroll = c.unroll;
  *threads = c.threads;
  *split = c.split;
  *order = c.order;
  return RAID6C_OK;
}

int raid6c_split_mask(int p, int vec) {
  const ZpPrimeEntry* e = zp_prime_entry(p);
  if (e == nullptr || !(vec == 1 || vec == 2 || vec == 4)) return 0;
  return e->split_mask[vec];
}

void raid6c_tune_clear(void) { clear_tuned(); }

int raid6c_autotune_n(int p, int k, size_t row_bytes, void* base, size_t strip_stride, size_t stripe_stride,
                      size_t nstripes, int op, const int32_t* erasures, int reps, void* stream, float* best_ms) {
  g_last_error.clear();
  if (op != 0 && op != 1) return fail(RAID6C_E_ARG, "op = %d must be 0 (encode) or 1 (recovery)", op);
  if (reps < 1 || reps > 1000) return fail(RAID6C_E_ARG, "reps must be in [1, 1000]");
  int rc = check_strided(p, k, row_bytes, base, strip_stride, stripe_stride, nstripes);
  if (rc != RAID6C_OK) return rc;
  if (op == 1 && (erasures == nullptr || ((uintptr_t)erasures & 3u) != 0))
    return fail(RAID6C_E_ARG, "erasures is NULL or not 4-byte aligned");
  const ZpPrimeEntry* e = zp_prime_entry(p);
  if (e == nullptr) return fail(RAID6C_E_UNSUPPORTED, "p = %d is not built", p);
  if (nstripes == 0) {
    if (best_ms) *best_ms = 0.f;
    return RAID6C_OK;
  }
  const hipStream_t s = (hipStream_t)stream;
  // One event before each timed launch and one after the last.
  std::vector<hipEvent_t> ev((size_t)reps + 1, nullptr);
  for (hipEvent_t& x : ev)
    if (hipEventCreate(&x) != hipSuccess) {
      for (hipEvent_t& y : ev)
        if (y != nullptr) (void)hipEventDestroy(y);
      return fail(RAID6C_E_HIP, "hipEventCreate failed");
    }
  const ZpKind kind = op == 0 ? KIND_ENCODE : KIND_RECOVER;
  const int slot = tune_slot(kind, k > p);
  const int bucket = row_bucket(row_bytes);
  ZpArgs a = strided_args(k, row_bytes, base, strip_stride, stripe_stride);
  a.erasures = op == 1 ? erasures : nullptr;
  ZpConfig best{0, 0, 0, 1};
  float best_t = 1e30f;
  // Every built configuration: (vec, unroll) with a work-group of 64, 128 or
  // 256 threads on separate column tiles, and split-K with 2 or 4 waves on
  // one tile.
  ZpConfig cands[9 * 5];
  int ncand = 0;
  for (int vec = 1; vec <= 4; vec *= 2)
    for (int unroll = 1; unroll <= 4; unroll *= 2) {
      if (!e->has(vec, unroll)) continue;
      for (int threads = 64; threads <= 256; threads *= 2) cands[ncand++] = ZpConfig{vec, unroll, threads, 1};
      for (int sp = 2; sp <= 4; sp *= 2)
        if (e->split_mask[vec] & sp) cands[ncand++] = ZpConfig{vec, unroll, 64 * sp, sp};
    }
  // Median time per launch of one configuration over `reps` launches timed
  // one by one (after one warm-up launch).
  std::vector<float> t((size_t)reps);
  auto time_cfg = [&](const ZpConfig& cfg, float* ms) {
    set_tuned(p, slot, bucket, cfg);
    int r2 = launch_zp(p, kind, a, nstripes, stream);
    if (r2 != RAID6C_OK) return r2;
    (void)hipEventRecord(ev[0], s);
    for (int r = 0; r < reps && r2 == RAID6C_OK; ++r) {
      r2 = launch_zp(p, kind, a, nstripes, stream);
      (void)hipEventRecord(ev[(size_t)r + 1], s);
    }
    if (r2 != RAID6C_OK) return r2;
    if (hipEventSynchronize(ev[(size_t)reps]) != hipSuccess) return fail(RAID6C_E_HIP, "hipEventSynchronize failed");
    for (int r = 0; r < reps; ++r) (void)hipEventElapsedTime(&t[(size_t)r], ev[(size_t)r], ev[(size_t)r + 1]);
    std::nth_element(t.begin(), t.begin() + reps / 2, t.end());
    *ms = t[(size_t)reps / 2];
    return RAID6C_OK;
  };
  float times[9 * 5];
  for (int ci = 0; ci < ncand && rc == RAID6C_OK; ++ci) {
    rc = time_cfg(cands[ci], &times[ci]);
    if (rc == RAID6C_OK && times[ci] < best_t) {
      best_t = times[ci];
      best = cands[ci];
    }
  }
  // The other work-group orders (XCD-chunked, stripes spread) for the
  // configurations within 5% of the best.
  const float cut = 1.05f * best_t;
  for (int ci = 0; ci < ncand && rc == RAID6C_OK; ++ci) {
    if (times[ci] > cut) continue;
    for (int order = 1; order <= 2 && rc == RAID6C_OK; ++order) {
      ZpConfig cfg = cands[ci];
      cfg.order = order;
      float ms = 0.f;
      rc = time_cfg(cfg, &ms);
      if (rc == RAID6C_OK && ms < best_t) {
        best_t = ms;
        best = cfg;
      }
    }
  }
  for (hipEvent_t& x : ev) (void)hipEventDestroy(x);
  if (rc != RAID6C_OK) return rc;
  set_tuned(p, slot, bucket, best);
  if (best_ms) *best_ms = best_t;
  return RAID6C_OK;
}

}  // extern "C"
