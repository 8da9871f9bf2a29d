// First-fit allocator of the server's arena (admission by HBM footprint):
// regions of [0, size), the lowest fitting offset first, neighbours
// coalesced on release.  Host-only bookkeeping; the bytes are device memory
// the caller owns.
#ifndef TN_SERVER_ARENA_HPP_
#define TN_SERVER_ARENA_HPP_

#include <cstddef>
#include <iterator>
#include <map>

namespace tn {

class Arena {
 public:
  explicit Arena(size_t size) {
    if (size) free_[0] = size;
  }
  // Reserves n bytes at the lowest offset with room; false if none has.
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += n;
        return true;
      }
    }
    return false;
  }
  // Returns a region obtained from alloc (same offset and size).
  void release(size_t off, size_t n) {
    used_ -= n;
    auto it = free_.emplace(off, n).first;
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
  size_t used() const { return used_; }
  // Free regions as (offset, size), ascending.
  const std::map<size_t, size_t>& free_regions() const { return free_; }

 private:
  size_t used_ = 0;
  std::map<size_t, size_t> free_;
};

}  // namespace tn

#endif  // TN_SERVER_ARENA_HPP_
