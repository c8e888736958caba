// syev3_pool.hpp -- first-fit allocator of byte ranges in the server's
// device pool (host-side bookkeeping only; no device calls).
#pragma once

#include <stddef.h>

#include <iterator>
#include <map>

namespace syev3 {

// First-fit allocator over [0, size) with coalescing frees.  alloc() takes
// the lowest-offset free range that fits; release() merges neighbours.
class PoolAllocator {
 public:
  explicit PoolAllocator(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t noff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        in_use_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    in_use_ -= bytes;
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
  size_t in_use() const { return in_use_; }
  size_t size() const { return size_; }

 private:
  size_t size_;
  size_t in_use_ = 0;
  std::map<size_t, size_t> free_;
};

}  // namespace syev3
