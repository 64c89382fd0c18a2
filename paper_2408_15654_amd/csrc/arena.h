// arena.h - host-side allocator of the batch workspace (plain C++, no HIP).
#ifndef LBM_ARENA_H
#define LBM_ARENA_H

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>

namespace lbm_host {

inline size_t arena_align(size_t v) { return (v + 255) / 256 * 256; }

// Allocator over a byte range of the caller's workspace: first fit from the
// bottom (the simulations' blocks) or last fit from the top (the batch's
// growing metadata); freed blocks coalesce with free neighbours.  Offsets
// and sizes are multiples of 256 bytes.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = arena_align(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t left = it->second - bytes, next = it->first + bytes;
      free_.erase(it);
      if (left) free_[next] = left;
      return true;
    }
    return false;
  }
  // Last fit, from the top of the range: for the batch's own growing
  // metadata, so it does not split the space simulations are admitted into.
  bool alloc_top(size_t bytes, size_t *off) {
    bytes = arena_align(bytes);
    for (auto it = free_.rbegin(); it != free_.rend(); ++it) {
      if (it->second < bytes) continue;
      it->second -= bytes;
      *off = it->first + it->second;
      if (it->second == 0) free_.erase(std::next(it).base());
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = arena_align(bytes);
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
  size_t largest() const {
    size_t m = 0;
    for (const auto &kv : free_) m = std::max(m, kv.second);
    return m;
  }

 private:
  std::map<size_t, size_t> free_;  // offset -> size
};

}  // namespace lbm_host

#endif
