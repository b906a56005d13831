// serve_sched.h — the serving scheduler's host-side policy, free of HIP so
// that it can be checked on its own: the first-fit device arena and the
// first-in first-out admission rule.  Not part of the public ABI.
#pragma once

#include <cstddef>
#include <deque>
#include <iterator>
#include <map>

namespace hr2 {

inline size_t round256(size_t n) { return (n + 255) & ~size_t(255); }

// First-fit allocator over [0, cap) in 256-byte units: free blocks are kept
// by offset and fully coalesced, so an allocation takes the lowest offset
// where enough contiguous free space starts.
class Arena {
 public:
  explicit Arena(size_t cap = 0) { reset(cap); }
  void reset(size_t cap) {
    free_.clear();
    cap_ = cap;
    used_ = 0;
    if (cap) free_[0] = cap;
  }
  bool alloc(size_t n, size_t *off) {
    n = round256(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n, start = it->first + n;
      free_.erase(it);
      if (rest) free_[start] = rest;
      used_ += n;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = round256(n);
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
  size_t cap() const { return cap_; }
  size_t free_blocks() const { return free_.size(); }

 private:
  std::map<size_t, size_t> free_;
  size_t cap_ = 0, used_ = 0;
};

// First-in first-out admission: admit the head of `pending` while its
// footprint (bytes_of) fits the arena and fewer than max_slots requests are
// admitted; stop at the first request that does not fit, so no request
// overtakes an older one.  on_admit(request, offset) runs for each admitted
// request, oldest first.  Returns the number admitted.
template <typename R, typename BytesOf, typename OnAdmit>
int admit_fifo(std::deque<R *> &pending, Arena &arena, int max_slots, int &n_admitted,
               BytesOf bytes_of, OnAdmit on_admit) {
  int k = 0;
  while (!pending.empty() && n_admitted < max_slots) {
    R *r = pending.front();
    size_t off = 0;
    if (!arena.alloc(bytes_of(r), &off)) break;
    ++n_admitted;
    ++k;
    pending.pop_front();
    on_admit(r, off);
  }
  return k;
}

}  // namespace hr2
