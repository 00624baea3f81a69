// Range allocator over one device arena (host-side bookkeeping only): the
// request server carves each admitted solve's state out of a fixed HBM
// budget and returns it when the solve leaves.  First fit over a free list
// ordered by offset, ranges aligned to `align` bytes, neighbours merged on
// free.  No device calls; unit-tested on the host.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace gm {

class RangePool {
 public:
  static constexpr size_t npos = ~size_t(0);

  RangePool(size_t bytes = 0, size_t align = 256) : align_(align) { reset(bytes); }

  void reset(size_t bytes) {
    free_.clear();
    cap_ = bytes / align_ * align_;
    used_ = 0;
    peak_ = 0;
    if (cap_) free_[0] = cap_;
  }

  static size_t round_up(size_t n, size_t a) { return (n + a - 1) / a * a; }

  // Offset of a free range of at least `bytes` (rounded up to the alignment),
  // or npos when no free range is large enough.
  size_t alloc(size_t bytes) {
    const size_t need = round_up(bytes ? bytes : 1, align_);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > need) free_[off + need] = len - need;
      used_ += need;
      if (used_ > peak_) peak_ = used_;
      return off;
    }
    return npos;
  }

  // Return a range obtained from alloc(bytes).
  void release(size_t off, size_t bytes) {
    const size_t len = round_up(bytes ? bytes : 1, align_);
    used_ -= len;
    auto next = free_.lower_bound(off);
    size_t start = off, size = len;
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        start = prev->first;
        size += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && off + len == next->first) {
      size += next->second;
      free_.erase(next);
    }
    free_[start] = size;
  }

  // Largest single range that alloc() could return now.
  size_t largest_free() const {
    size_t m = 0;
    for (auto &f : free_)
      if (f.second > m) m = f.second;
    return m;
  }

  size_t capacity() const { return cap_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t fragments() const { return free_.size(); }

 private:
  size_t align_, cap_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length, disjoint, not adjacent
};

}  // namespace gm
