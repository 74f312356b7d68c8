// dev_arena.hpp -- a device-memory arena: one hipMalloc'd region handed out in
// 256-byte-aligned pieces (first fit, neighbours coalesced on release).  A
// serving process allocates the arena once at its HBM budget, so requests
// taking and returning memory never call hipMalloc or hipFree while other
// requests' kernels run.  Thread-safe.
#pragma once
#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>
#include <mutex>

namespace cptr {

class DevArena {
 public:
  static constexpr size_t kAlign = 256;
  static size_t round(size_t bytes) { return (bytes + kAlign - 1) / kAlign * kAlign; }

  // `base` must be kAlign-aligned and hold `size` bytes (owned by the caller)
  void init(void* base, size_t size) {
    std::lock_guard<std::mutex> g(mu_);
    base_ = static_cast<char*>(base);
    size_ = size / kAlign * kAlign;
    free_.clear();
    used_.clear();
    if (size_ > 0) free_[0] = size_;
    in_use_ = 0;
  }
  // nullptr when no free piece is large enough
  void* alloc(size_t bytes) {
    const size_t n = round(bytes == 0 ? 1 : bytes);
    std::lock_guard<std::mutex> g(mu_);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[off + n] = len - n;
      used_[off] = n;
      in_use_ += n;
      return base_ + off;
    }
    return nullptr;
  }
  // false when p is not a live piece of this arena
  bool release(void* p) {
    std::lock_guard<std::mutex> g(mu_);
    const size_t off = static_cast<size_t>(static_cast<char*>(p) - base_);
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    size_t start = off, len = u->second;
    used_.erase(u);
    in_use_ -= len;
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
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
  size_t in_use() const {
    std::lock_guard<std::mutex> g(mu_);
    return in_use_;
  }
  size_t largest_free() const {
    std::lock_guard<std::mutex> g(mu_);
    size_t m = 0;
    for (const auto& f : free_) m = f.second > m ? f.second : m;
    return m;
  }
  size_t size() const { return size_; }

 private:
  mutable std::mutex mu_;
  char* base_ = nullptr;
  size_t size_ = 0;
  size_t in_use_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  std::map<size_t, size_t> used_;  // offset -> length
};

}  // namespace cptr
