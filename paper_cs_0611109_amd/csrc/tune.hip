// tune.hip -- launch-configuration choice (built-in rule plus a tuning table).
#include "tune.h"

#include <stdlib.h>

#include <atomic>

namespace raid6c {

namespace {

constexpr int kBuckets = 31;
// Packed (order << 24 | split << 20 | vec << 16 | unroll << 12 | threads), 0 = no entry;
// [p][slot][bucket] (slot: tune_slot).
std::atomic<uint32_t> g_table[kMaxPrime + 1][kTuneSlots][kBuckets];

int env_int(const char* name) {
  const char* s = getenv(name);
  return s ? atoi(s) : 0;
}

bool valid(const ZpPrimeEntry& e, const ZpConfig& c) { return e.has(c); }

uint32_t pack(const ZpConfig& c) {
  return ((uint32_t)c.order << 24) | ((uint32_t)c.split << 20) | ((uint32_t)c.vec << 16) |
         ((uint32_t)c.unroll << 12) | (uint32_t)c.threads;
}

ZpConfig unpack(uint32_t t) {
  return ZpConfig{(int)((t >> 16) & 0xF), (int)((t >> 12) & 0xF), (int)(t & 0xFFF), (int)((t >> 20) & 0xF),
                  (int)((t >> 24) & 0xF)};
}

}  // namespace

int row_bucket(uint64_t row_bytes) {
  int b = 0;
  while (b < kBuckets - 1 && (row_bytes >> (b + 1)) != 0) ++b;
  return b;
}

bool set_tuned(int p, int slot, int bucket, ZpConfig cfg) {
  if (p < 3 || p > kMaxPrime || bucket < 0 || bucket >= kBuckets) return false;
  if (slot < 0 || slot >= kTuneSlots) return false;
  g_table[p][slot][bucket].store(pack(cfg));
  return true;
}

void clear_tuned() {
  for (auto& a : g_table)
    for (auto& b : a)
      for (auto& c : b) c.store(0);
}

ZpConfig default_config(const ZpPrimeEntry& e, ZpKind kind, uint64_t row_bytes) {
  (void)kind;
  // Pick the (vec, unroll) pair that keeps the most load bytes in flight per
  // compute unit: registers per thread ~ (2p-1)*vec accumulators + a batch of
  // unroll*(p-1)*vec loads + ~24 for addresses and temporaries; a SIMD holds
  // floor(512 / registers) waves, at most 8.
  const int p = e.p;
  ZpConfig best{0, 0, 64, 1};
  long best_score = -1;
  for (int vec = 1; vec <= 4; vec *= 2) {
    for (int unroll = 1; unroll <= 4; unroll *= 2) {
      if (!e.has(vec, unroll)) continue;
      const int regs = (2 * p - 1) * vec + unroll * (p - 1) * vec + 24;
      int waves = 512 / regs;
      if (waves > 8) waves = 8;
      // Lanes past the end of a short row do no work: discount them.
      const uint64_t tile = 64ull * vec * 4;
      const double used = row_bytes >= tile ? 1.0 : (double)row_bytes / (double)tile;
      const long score = (long)(waves * unroll * (p - 1) * vec * used * 1000.0);
      // On a tie the larger batch of loads wins (it measured faster: four
      // strips at one wave per SIMD beat two at two waves for the large p).
      if (score >= best_score) {
        best_score = score;
        best = ZpConfig{vec, unroll, 64, 1};
      }
    }
  }
  // Work-groups of up to 256 threads, as many as a row has lanes for: 256
  // measured 3-8% faster than 64 wherever the row is long enough.
  const uint64_t lanes = (row_bytes + best.vec * 4 - 1) / (best.vec * 4);
  best.threads = lanes > 128 ? 256 : lanes > 64 ? 128 : 64;
  // Several waves per column tile (split-K) with two dwords per lane, where
  // their partials fit in LDS: fewer stripes in flight at once, which
  // measured fastest on MI355X for the primes that allow it (p <= 31).
  if (row_bytes >= 64 * 2 * 4) {
    if (e.split_mask[2] & 4) return ZpConfig{2, 1, 256, 4};
    if (e.split_mask[2] & 2) return ZpConfig{2, 1, 128, 2};
  }
  // Larger primes: two dwords per lane, one strip per batch, when the row is
  // a whole number of such tiles (the largest work-group whose tile divides
  // the row): p = 37..61 measured 78-80% against 72-76% for the pair chosen
  // above.  A row with a ragged last tile keeps the pair above (a mostly
  // empty tile costs a whole work-group).
  if (e.has(2, 1) && row_bytes % (64 * 2 * 4) == 0) {
    const int threads = row_bytes % (256 * 2 * 4) == 0 ? 256 : row_bytes % (128 * 2 * 4) == 0 ? 128 : 64;
    return ZpConfig{2, 1, threads, 1};
  }
  return best;
}

ZpConfig choose_config(const ZpPrimeEntry& e, int slot, uint64_t row_bytes) {
  // Explicit override (used by tuning sweeps).
  static const int env_vec = env_int("RAID6C_ZP_VEC");
  static const int env_unroll = env_int("RAID6C_ZP_UNROLL");
  static const int env_threads = env_int("RAID6C_ZP_THREADS");
  static const int env_split = env_int("RAID6C_ZP_SPLIT");
  static const int env_order = env_int("RAID6C_ZP_ORDER");
  if (env_vec != 0 && env_threads != 0) {
    const ZpConfig c{env_vec, env_unroll ? env_unroll : 1, env_threads, env_split ? env_split : 1, env_order};
    if (valid(e, c)) return c;
  }
  const uint32_t t = g_table[e.p][slot][row_bucket(row_bytes)].load();
  if (t != 0) {
    const ZpConfig c = unpack(t);
    if (valid(e, c)) return c;
  }
  return default_config(e, (ZpKind)(slot & 1), row_bytes);
}

static std::atomic<uint32_t> g_rs_override{0};  // vec<<16 | unroll<<12 | threads, 0 = none

bool set_rs_override(int vec, int unroll, int threads) {
  if (vec == 0 && unroll == 0 && threads == 0) {
    g_rs_override.store(0);
    return true;
  }
  if ((vec != 1 && vec != 2 && vec != 4) || (unroll != 1 && unroll != 4 && unroll != 8) ||
      (threads != 64 && threads != 128 && threads != 256))
    return false;
  g_rs_override.store(((uint32_t)vec << 16) | ((uint32_t)unroll << 12) | (uint32_t)threads);
  return true;
}

RsConfig choose_rs_config(uint64_t strip_bytes, bool recovery) {
  const uint32_t o = g_rs_override.load();
  if (o != 0) return RsConfig{(int)(o >> 16), (int)((o >> 12) & 15u), (int)(o & 0xFFFu)};
  static const int env_vec = env_int("RAID6C_RS_VEC");
  static const int env_unroll = env_int("RAID6C_RS_UNROLL");
  static const int env_threads = env_int("RAID6C_RS_THREADS");
  if ((env_vec == 1 || env_vec == 2 || env_vec == 4) && (env_unroll == 1 || env_unroll == 4 || env_unroll == 8) &&
      (env_threads == 64 || env_threads == 128 || env_threads == 256))
    return RsConfig{env_vec, env_unroll, env_threads};
  // Measured on MI355X (12 data strips of 48 KiB): encode is fastest with one
  // dword per thread and 4 strips in flight (about 80% of HBM peak); the
  // two-data recovery multiplies by two field constants per byte and needs
  // the wider vectors to stay near the memory rate.
  const int vec = recovery ? 4 : 1;
  const int cap = recovery ? 256 : 128;
  int threads = 64;
  while (threads < cap && (uint64_t)threads * vec * 4 < strip_bytes) threads *= 2;
  return RsConfig{vec, 4, threads};
}

}  // namespace raid6c
