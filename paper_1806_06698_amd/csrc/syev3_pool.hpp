// syev3_pool.hpp -- first-fit allocator of byte ranges in the server's
// device pool (host-side bookkeeping only; no device calls).
#pragma once

#include <stddef.h>

#include <iterator>
#include <map>
#include <utility>

namespace syev3 {

// First-fit allocator over [0, size) with coalescing frees.  alloc() takes
// the lowest-offset free range that fits; release() merges neighbours.
//
// Exception safety: the free list is a std::map, whose node allocation can
// throw std::bad_alloc.  Both operations give the strong guarantee: a throw
// leaves the allocator exactly as it was (no range lost or double-counted).
//  * alloc() inserts the remainder of a split range before erasing the
//    range it came from (inserting is the only step that allocates);
//  * release() merges into a neighbour in place, or moves the following
//    range's node to the new start (node handles: no allocation), and
//    allocates a node only for a range with no free neighbour.
class PoolAllocator {
 public:
  explicit PoolAllocator(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t start = it->first;
        const size_t rest = it->second - bytes;
        if (rest) free_.emplace_hint(std::next(it), start + bytes, rest);  // may throw
        free_.erase(it);
        in_use_ += bytes;
        *off = start;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto nx = free_.lower_bound(off);  // first free range after the block
    const bool join_next = nx != free_.end() && off + bytes == nx->first;
    auto pv = nx == free_.begin() ? free_.end() : std::prev(nx);
    const bool join_prev = pv != free_.end() && pv->first + pv->second == off;
    if (join_prev) {
      pv->second += bytes;
      if (join_next) {
        pv->second += nx->second;
        free_.erase(nx);
      }
    } else if (join_next) {
      auto node = free_.extract(nx);
      node.key() = off;
      node.mapped() += bytes;
      free_.insert(std::move(node));
    } else {
      free_.emplace_hint(nx, off, bytes);  // may throw
    }
    in_use_ -= bytes;
  }
  size_t in_use() const { return in_use_; }
  size_t size() const { return size_; }
  // The free ranges (offset -> length), for tests.
  const std::map<size_t, size_t>& free_ranges() const { return free_; }

 private:
  size_t size_;
  size_t in_use_ = 0;
  std::map<size_t, size_t> free_;
};

}  // namespace syev3
