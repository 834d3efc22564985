// Host-only pieces of the server, kept free of HIP so that they can be
// built and tested on their own (with sanitizers) on any host: the
// first-fit arena allocator and the admission rule for a round.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <iterator>
#include <map>

namespace ss {

constexpr size_t kArenaAlign = 256;
inline size_t arena_round_up(size_t x) { return (x + kArenaAlign - 1) & ~(kArenaAlign - 1); }

// First-fit allocator over [0, size) in 256-byte units, with coalescing of
// freed neighbours.  Offsets are relative to the arena's start.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    size_ = size & ~(kArenaAlign - 1);
    if (size_) free_[0] = size_;
    used_ = 0;
  }
  // Lowest-addressed free block of at least `bytes` (rounded up to 256).
  bool alloc(size_t bytes, size_t* off) {
    bytes = arena_round_up(bytes ? bytes : kArenaAlign);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  // Returns a block obtained from alloc (same offset and size).
  void release(size_t off, size_t bytes) {
    bytes = arena_round_up(bytes ? bytes : kArenaAlign);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }
  size_t free_blocks() const { return free_.size(); }
  size_t largest_free() const {
    size_t best = 0;
    for (const auto& kv : free_) best = kv.second > best ? kv.second : best;
    return best;
  }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0, used_ = 0;
};

// Admission of a round: the longest prefix of the first `n` waiting
// requests whose workspace and outputs both fit the arena now.  round_bytes(k,
// &ws, &out) gives the two sizes of a round of the first k requests and
// returns false when such a round cannot exist at all (e.g. too many pairs).
// On success the two blocks are allocated and k is returned; 0 when not even
// the first request fits now.  *never_fits is set when the first request
// alone could not fit even an empty arena (its round cannot exist, or its
// two blocks exceed the arena's size).
template <typename RoundBytes>
uint32_t admit_prefix(Arena& arena, uint32_t n, RoundBytes&& round_bytes, size_t* ws_off, size_t* ws_bytes,
                      size_t* out_off, size_t* out_bytes, bool* never_fits) {
  *never_fits = false;
  for (uint32_t k = n; k >= 1; --k) {
    size_t ws = 0, out = 0;
    const bool exists = round_bytes(k, &ws, &out);
    if (exists && arena.alloc(ws, ws_off)) {
      if (arena.alloc(out, out_off)) {
        *ws_bytes = ws;
        *out_bytes = out;
        return k;
      }
      arena.release(*ws_off, ws);
    }
    if (k == 1) *never_fits = !exists || arena_round_up(ws) + arena_round_up(out) > arena.size();
  }
  return 0;
}

}  // namespace ss
