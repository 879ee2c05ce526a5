// Randomised checks of the request server's host bookkeeping
// (paper_cs_0611109_amd/csrc/stripe_index.h), built with the host compiler:
//  * StripeIndex against std::unordered_map under random inserts, erasures
//    and lookups (sequential, strided and random ids; several table sizes);
//  * ring_fit in a first-in-first-out store: every placement lies inside
//    the store and overlaps no resident stripe, and an empty store takes any
//    stripe that is not larger than it.
// Prints "ok" and exits 0, or names the first failure and exits 1.
#include <stdio.h>
#include <stdlib.h>

#include <deque>
#include <random>
#include <unordered_map>
#include <vector>

#include "../../paper_cs_0611109_amd/csrc/stripe_index.h"

using raid6c::ring_fit;
using raid6c::StripeIndex;

static int fail(const char* what, unsigned long long a, unsigned long long b) {
  printf("FAIL %s (%llu, %llu)\n", what, a, b);
  return 1;
}

static int check_index(uint64_t seed, int pattern, int ops) {
  std::mt19937_64 g(seed);
  StripeIndex<int> idx(16);
  std::unordered_map<uint64_t, int*> ref;
  std::vector<int> vals(1);
  std::vector<uint64_t> keys;
  uint64_t next = 0;
  for (int op = 0; op < ops; ++op) {
    const unsigned r = (unsigned)(g() % 10);
    if (r < 5 || keys.empty()) {
      uint64_t k = pattern == 0 ? next++ : pattern == 1 ? (next++) * 4096 : g();
      if (ref.count(k)) continue;
      int* v = reinterpret_cast<int*>(0x1000 + 16 * (uintptr_t)(op + 1));
      idx.insert(k, v);
      ref[k] = v;
      keys.push_back(k);
    } else if (r < 8) {
      const size_t j = g() % keys.size();
      const uint64_t k = keys[j];
      const bool had = idx.erase(k);
      if (!had) return fail("erase of a present key", k, op);
      ref.erase(k);
      keys[j] = keys.back();
      keys.pop_back();
      if (idx.erase(k)) return fail("second erase", k, op);
    } else {
      const uint64_t k = (g() & 1) && !keys.empty() ? keys[g() % keys.size()] : g();
      auto it = ref.find(k);
      int* want = it == ref.end() ? nullptr : it->second;
      if (idx.find(k) != want) return fail("lookup", k, op);
    }
    if (idx.size() != ref.size()) return fail("size", idx.size(), ref.size());
  }
  for (auto& kv : ref)
    if (idx.find(kv.first) != kv.second) return fail("final lookup", kv.first, 0);
  return 0;
}

struct Span {
  uint64_t off, bytes;
};

static int check_ring(uint64_t seed, uint64_t end, uint64_t max_need, int ops) {
  std::mt19937_64 g(seed);
  std::deque<Span> fifo;
  uint64_t head = 0;
  for (int op = 0; op < ops; ++op) {
    const uint64_t need = 1 + g() % max_need;
    if (need > end) {
      uint64_t off;
      if (ring_fit(head, 0, true, need, end, &off)) return fail("oversized stripe placed", need, end);
      continue;
    }
    for (;;) {
      uint64_t off = 0;
      const bool fits = ring_fit(head, fifo.empty() ? 0 : fifo.front().off, fifo.empty(), need, end, &off);
      if (fits) {
        if (off + need > end) return fail("placement past the end", off, need);
        for (const Span& sp : fifo)
          if (off < sp.off + sp.bytes && sp.off < off + need) return fail("overlap", off, sp.off);
        fifo.push_back(Span{off, need});
        head = off + need;
        break;
      }
      if (fifo.empty()) return fail("empty store refused a stripe", need, end);
      fifo.pop_front();
    }
    // Sometimes retire stripes early, oldest first, as evictions do.
    if (g() % 7 == 0)
      for (int n = (int)(g() % 3); n > 0 && !fifo.empty(); --n) fifo.pop_front();
  }
  return 0;
}

int main() {
  for (int pattern = 0; pattern < 3; ++pattern)
    for (uint64_t seed = 1; seed <= 4; ++seed)
      if (check_index(seed * 7919 + pattern, pattern, 40000)) return 1;
  const uint64_t ends[] = {4096, 100000, 1 << 20};
  for (uint64_t end : ends)
    for (uint64_t seed = 1; seed <= 4; ++seed) {
      if (check_ring(seed, end, end / 3, 20000)) return 1;
      if (check_ring(seed + 100, end, end, 20000)) return 1;
      if (check_ring(seed + 200, end, end / 50 + 1, 20000)) return 1;
    }
  printf("ok\n");
  return 0;
}
