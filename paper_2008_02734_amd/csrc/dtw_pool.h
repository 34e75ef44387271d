// First-fit allocator over one device memory range (the serving pool):
// offsets and sizes only, no device calls, so it is unit-tested on the host.
// Blocks are aligned to 256 bytes; freed blocks merge with their neighbours.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace dtw {

class PoolAllocator {
 public:
  static constexpr size_t kAlign = 256;

  explicit PoolAllocator(size_t bytes = 0) { reset(bytes); }

  void reset(size_t bytes) {
    free_.clear();
    used_.clear();
    size_ = bytes & ~(kAlign - 1);
    if (size_) free_[0] = size_;
  }

  // Offset of a new block of at least `bytes`, or SIZE_MAX when none fits.
  size_t alloc(size_t bytes) {
    const size_t need = round_up(bytes == 0 ? 1 : bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > need) free_[off + need] = len - need;
      used_[off] = need;
      return off;
    }
    return SIZE_MAX;
  }

  // Returns false for an offset that is not an allocated block.
  bool release(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    size_t start = off, len = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && start + len == next->first) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
    return true;
  }

  size_t largest_free() const {
    size_t best = 0;
    for (const auto& kv : free_) best = kv.second > best ? kv.second : best;
    return best;
  }
  size_t free_bytes() const {
    size_t t = 0;
    for (const auto& kv : free_) t += kv.second;
    return t;
  }
  size_t size() const { return size_; }
  size_t n_used() const { return used_.size(); }
  static size_t round_up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

 private:
  size_t size_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  std::map<size_t, size_t> used_;  // offset -> length
};

}  // namespace dtw
