// tune.h -- launch-configuration choice for the kernels of libraid6c.
#pragma once

#include <stdint.h>

#include "raid6c_internal.h"

namespace raid6c {

struct RsConfig {
  int vec;      // dwords per thread: 1, 2 or 4
  int unroll;   // strips whose loads are issued together: 1, 4 or 8
  int threads;  // 64, 128 or 256
};

// Tuning-table slot of an operation: 0 encode, 1 recovery, 2 and 3 the same
// for stripes with the extended Q parity (k > p), whose best configurations
// differ from the plain code's.
inline int tune_slot(ZpKind kind, bool ext) { return (int)kind + (ext ? 2 : 0); }
constexpr int kTuneSlots = 4;

// Configuration for a Z_p kernel: a tuned entry when one has been recorded
// for (p, slot, row-size bucket), else the built-in rule.
ZpConfig choose_config(const ZpPrimeEntry& e, int slot, uint64_t row_bytes);

// The built-in rule alone.
ZpConfig default_config(const ZpPrimeEntry& e, ZpKind kind, uint64_t row_bytes);

// Configuration for the GF(256) comparison kernel: the override when one is
// set, else the built-in rule (environment variables first).
RsConfig choose_rs_config(uint64_t strip_bytes, bool recovery);
bool set_rs_override(int vec, int unroll, int threads);  // (0, 0, 0) clears

// Row-size bucket used by the tuning table: floor(log2(row_bytes)), 0..30.
int row_bucket(uint64_t row_bytes);

// Record / forget a tuned configuration (the autotuner's output).
bool set_tuned(int p, int slot, int bucket, ZpConfig cfg);
void clear_tuned();

}  // namespace raid6c
