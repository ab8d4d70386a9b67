// First-fit allocator of the serving loop's output arena: byte ranges of
// [0, size), free neighbours coalesced.  Host logic only (no HIP), so that it
// is also built and checked on its own.
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace zg {

class Arena {
 public:
  void init(uint64_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  // The lowest free range of at least `bytes`; false when none is large enough.
  bool alloc(uint64_t bytes, uint64_t *off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const uint64_t rest = it->second - bytes, start = it->first + bytes;
      free_.erase(it);
      if (rest) free_[start] = rest;
      return true;
    }
    return false;
  }
  // Returns [off, off + bytes), which alloc handed out, and merges it with
  // free neighbours.
  void release(uint64_t off, uint64_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  // Free ranges (offset -> length), for checks.
  const std::map<uint64_t, uint64_t> &free_ranges() const { return free_; }

 private:
  std::map<uint64_t, uint64_t> free_;
};

}  // namespace zg
