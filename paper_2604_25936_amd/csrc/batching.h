// Host-side scheduling pieces of the serving loop (server.cpp), free of any
// device code so that they can be unit-tested on the CPU under sanitizers:
// the first-fit arena that admits requests by device bytes, and the choice
// of which admitted requests form the next batch.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace sand {

// First-fit allocator over offsets [0, size) of one device allocation.
// Freed ranges coalesce with free neighbours; `used` and `peak` count bytes.
class Arena {
 public:
  void init(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    used = peak = 0;
  }
  bool alloc(size_t n, size_t* off) {
    if (n == 0) return false;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n, at = it->first + n;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used += n;
      peak = std::max(peak, used);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    if (n == 0) return;
    used -= n;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }
  // Free ranges in offset order (tests).
  std::vector<std::pair<size_t, size_t>> free_ranges() const {
    return std::vector<std::pair<size_t, size_t>>(free_.begin(), free_.end());
  }
  size_t used = 0, peak = 0;

 private:
  std::map<size_t, size_t> free_;   // offset -> size of each free range
};

// Admit pending requests first-in first-out while their bytes fit the
// arena: nothing overtakes the head of the queue. R has members `bytes`
// and `off`. Returns how many were admitted.
template <class R>
int admit_fifo(std::deque<R*>& pending, std::deque<R*>& admitted, Arena& arena) {
  int k = 0;
  while (!pending.empty()) {
    R* r = pending.front();
    size_t off;
    if (!arena.alloc(r->bytes, &off)) break;
    r->off = off;
    admitted.push_back(r);
    pending.pop_front();
    ++k;
  }
  return k;
}

// The next batch: admitted requests that share the head's key (padded
// width and activation: one kernel instantiation), in order, while their
// points stay within `point_cap` (the head always goes) and at most
// `max_reqs` of them. Taken requests leave `admitted`. R has `n`; key(R*)
// returns a comparable value.
template <class R, class Key>
std::vector<R*> take_batch(std::deque<R*>& admitted, int64_t point_cap, int max_reqs, Key key) {
  std::vector<R*> out;
  if (admitted.empty()) return out;
  const auto k0 = key(admitted.front());
  int64_t points = 0;
  for (auto it = admitted.begin(); it != admitted.end() && (int)out.size() < max_reqs;) {
    const bool fits = out.empty() || points + (*it)->n <= point_cap;
    if (key(*it) == k0 && fits) {
      points += (*it)->n;
      out.push_back(*it);
      it = admitted.erase(it);
    } else {
      ++it;
    }
  }
  return out;
}

}  // namespace sand
