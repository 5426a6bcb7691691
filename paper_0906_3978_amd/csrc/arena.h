// First-fit arena over one device allocation (host bookkeeping only: no
// device calls), in 256-byte granules.  The serving loop allocates every
// request's buffers from it, so admission is an allocation against the
// budget.  Thread-safe.
#pragma once

#include <algorithm>
#include <cstddef>
#include <map>
#include <mutex>

namespace wf {

struct Arena {
  char* base = nullptr;
  size_t size = 0;
  std::mutex mu;
  std::map<size_t, size_t> free_;   // offset -> bytes
  std::map<size_t, size_t> used_;   // offset -> bytes
  size_t in_use = 0, peak = 0;

  void init(void* p, size_t n) {
    base = static_cast<char*>(p);
    size = n & ~size_t(255);
    free_.clear();
    used_.clear();
    free_[0] = size;
    in_use = peak = 0;
  }
  void* get(size_t bytes) {
    bytes = (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
    std::lock_guard<std::mutex> g(mu);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, left = it->second - bytes;
      free_.erase(it);
      if (left) free_[off + bytes] = left;
      used_[off] = bytes;
      in_use += bytes;
      peak = std::max(peak, in_use);
      return base + off;
    }
    return nullptr;
  }
  void put(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu);
    const size_t off = static_cast<char*>(p) - base;
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t len = u->second;
    used_.erase(u);
    in_use -= len;
    size_t start = off;
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && nx->first == off + len) {
      len += nx->second;
      free_.erase(nx);
    }
    auto pv = free_.lower_bound(off);
    if (pv != free_.begin()) {
      --pv;
      if (pv->first + pv->second == off) {
        start = pv->first;
        len += pv->second;
        free_.erase(pv);
      }
    }
    free_[start] = len;
  }
};


}  // namespace wf
