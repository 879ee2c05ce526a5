// stripe_index.h -- host-side bookkeeping of the request server's stripe
// store (host code only; not thread-safe: the server calls it under its
// lock).
//
// StripeIndex maps a stripe id to its resident record: open addressing with
// linear probing, at most half full, erasure by backward shift (no
// tombstones), so a lookup touches one or two cache lines and neither
// insertion nor erasure allocates (except to double the table).
//
// ring_fit places a stripe in the store, a ring of bytes [0, end).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace raid6c {

template <typename V>
class StripeIndex {
 public:
  explicit StripeIndex(size_t capacity = 1024) { rehash(round_pow2(capacity < 16 ? 16 : capacity)); }

  size_t size() const { return n_; }

  // The value stored under `key`, or nullptr.
  V* find(uint64_t key) const {
    for (size_t i = home(key);; i = (i + 1) & mask_) {
      if (val_[i] == nullptr) return nullptr;
      if (key_[i] == key) return val_[i];
    }
  }

  // Store `v` (not nullptr) under `key`, which must not be present.
  void insert(uint64_t key, V* v) {
    if (2 * (n_ + 1) > key_.size()) rehash(2 * key_.size());
    size_t i = home(key);
    while (val_[i] != nullptr) i = (i + 1) & mask_;
    key_[i] = key;
    val_[i] = v;
    ++n_;
  }

  // Remove `key`; returns whether it was present.  Later entries of the probe
  // run move back into the hole when their home position allows it, so every
  // entry stays reachable from its home without tombstones.
  bool erase(uint64_t key) {
    size_t i = home(key);
    while (val_[i] != nullptr && key_[i] != key) i = (i + 1) & mask_;
    if (val_[i] == nullptr) return false;
    val_[i] = nullptr;
    --n_;
    for (size_t j = (i + 1) & mask_; val_[j] != nullptr; j = (j + 1) & mask_) {
      const size_t h = home(key_[j]);
      // Entry j may fill the hole at i unless its home lies cyclically in (i, j].
      const bool stays = i <= j ? (h > i && h <= j) : (h > i || h <= j);
      if (stays) continue;
      key_[i] = key_[j];
      val_[i] = val_[j];
      val_[j] = nullptr;
      i = j;
    }
    return true;
  }

 private:
  static size_t round_pow2(size_t x) {
    size_t c = 1;
    while (c < x) c <<= 1;
    return c;
  }
  // A 64-bit mixing step (xorshift-multiply), so that sequential ids spread.
  size_t home(uint64_t k) const {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    return (size_t)k & mask_;
  }
  void rehash(size_t cap) {
    std::vector<uint64_t> old_key;
    std::vector<V*> old_val;
    old_key.swap(key_);
    old_val.swap(val_);
    key_.assign(cap, 0);
    val_.assign(cap, nullptr);
    mask_ = cap - 1;
    n_ = 0;
    for (size_t i = 0; i < old_val.size(); ++i)
      if (old_val[i] != nullptr) insert(old_key[i], old_val[i]);
  }

  std::vector<uint64_t> key_;
  std::vector<V*> val_;
  size_t mask_ = 0;
  size_t n_ = 0;
};

// Stripes are placed at the head, moving forward (back to offset 0 when the
// rest of the store is too short), and evicted oldest first, so the resident
// ones always cover one arc of the ring: from the oldest one's offset `tail`
// to `head`, past the end of the store at most once.  Free space is the rest.
// Returns whether `need` bytes fit without evicting anything, and where.
inline bool ring_fit(uint64_t head, uint64_t tail, bool empty, uint64_t need, uint64_t end, uint64_t* off) {
  *off = head + need <= end ? head : 0;
  if (need > end) return false;
  if (empty) return true;
  if (head > tail) return *off == head || need <= tail;    // occupied [tail, head)
  if (head < tail) return *off == head && head + need <= tail;  // occupied [tail, ..) and [0, head)
  return false;                                            // the arc is the whole ring
}

}  // namespace raid6c
