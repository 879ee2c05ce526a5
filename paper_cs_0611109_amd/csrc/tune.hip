// tune.hip -- launch-configuration choice (built-in rule plus a tuning table).
#include "tune.h"

#include <stdlib.h>

#include <atomic>
#include <mutex>

namespace raid6c {

namespace {

constexpr int kBuckets = 31;
// Packed (vec << 16 | threads), 0 = no entry; index [p][kind][bucket].
std::atomic<uint32_t> g_table[kMaxPrime + 1][2][kBuckets];

int env_int(const char* name) {
  const char* s = getenv(name);
  return s ? atoi(s) : 0;
}

bool valid(const ZpConfig& c, int vec_mask) {
  return (c.vec == 1 || c.vec == 2 || c.vec == 4) && (vec_mask & c.vec) &&
         (c.threads == 64 || c.threads == 128 || c.threads == 256);
}

}  // namespace

int row_bucket(uint64_t row_bytes) {
  int b = 0;
  while (b < kBuckets - 1 && (row_bytes >> (b + 1)) != 0) ++b;
  return b;
}

bool set_tuned(int p, ZpKind kind, int bucket, ZpConfig cfg) {
  if (p < 3 || p > kMaxPrime || bucket < 0 || bucket >= kBuckets) return false;
  if (!(cfg.threads == 64 || cfg.threads == 128 || cfg.threads == 256)) return false;
  if (!(cfg.vec == 1 || cfg.vec == 2 || cfg.vec == 4)) return false;
  g_table[p][kind][bucket].store(((uint32_t)cfg.vec << 16) | (uint32_t)cfg.threads);
  return true;
}

void clear_tuned() {
  for (auto& a : g_table)
    for (auto& b : a)
      for (auto& c : b) c.store(0);
}

ZpConfig choose_config(int p, ZpKind kind, uint64_t row_bytes, int vec_mask) {
  // Explicit override (used by tuning sweeps).
  static const int env_vec = env_int("RAID6C_ZP_VEC");
  static const int env_threads = env_int("RAID6C_ZP_THREADS");
  ZpConfig c{0, 0};
  if (env_vec != 0 && env_threads != 0) {
    c = ZpConfig{env_vec, env_threads};
    if (valid(c, vec_mask)) return c;
  }
  const uint32_t t = g_table[p][kind][row_bucket(row_bytes)].load();
  if (t != 0) {
    c = ZpConfig{(int)(t >> 16), (int)(t & 0xFFFF)};
    if (valid(c, vec_mask)) return c;
  }
  // Built-in rule: vector width by register budget ((2p-1)*vec dwords of
  // accumulators), then the smallest group that spans the row, capped at 256.
  int vec = (p <= 7) ? 4 : (p <= 23) ? 2 : 1;
  while (!(vec_mask & vec)) vec >>= 1;
  int threads = 64;
  while (threads < 256 && (uint64_t)threads * vec * 4 < row_bytes) threads *= 2;
  return ZpConfig{vec, threads};
}

RsConfig choose_rs_config(uint64_t strip_bytes) {
  static const int env_vec = env_int("RAID6C_RS_VEC");
  static const int env_threads = env_int("RAID6C_RS_THREADS");
  if ((env_vec == 1 || env_vec == 2 || env_vec == 4) &&
      (env_threads == 64 || env_threads == 128 || env_threads == 256))
    return RsConfig{env_vec, env_threads};
  int threads = 64;
  while (threads < 256 && (uint64_t)threads * 16 < strip_bytes) threads *= 2;
  return RsConfig{4, threads};
}

}  // namespace raid6c
