// range_alloc.h - first-fit allocator of ranges in [0, capacity), used by
// the server for device bytes and component slots (admission by memory).
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace mpld {

// First-fit over a free list kept sorted by offset; released ranges merge
// with free neighbours, so an empty allocator is always one free range.
class RangeAlloc {
 public:
  void reset(int64_t cap) {
    cap_ = cap;
    used_ = 0;
    free_.clear();
    if (cap > 0) free_[0] = cap;
  }
  int64_t alloc(int64_t len, int64_t align) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      const int64_t beg = it->first, end = it->first + it->second;
      const int64_t start = (beg + align - 1) / align * align;
      if (start + len > end) continue;
      free_.erase(it);
      if (start > beg) free_[beg] = start - beg;
      if (start + len < end) free_[start + len] = end - (start + len);
      used_ += len;
      return start;
    }
    return -1;
  }
  void release(int64_t off, int64_t len) {
    if (len <= 0) return;
    used_ -= len;
    auto it = free_.emplace(off, len).first;
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
  int64_t used() const { return used_; }
  int64_t capacity() const { return cap_; }

 private:
  std::map<int64_t, int64_t> free_;
  int64_t cap_ = 0, used_ = 0;
};

}  // namespace mpld
