// Randomised check of DevArena over a host buffer: pieces never overlap, stay
// aligned and inside the region, the byte count matches, and once everything
// is released the free list is one piece again (coalescing).
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "dev_arena.hpp"

int main() {
  const size_t size = 1 << 20;
  std::vector<unsigned char> mem(size + cptr::DevArena::kAlign);
  const size_t mis = reinterpret_cast<uintptr_t>(mem.data()) % cptr::DevArena::kAlign;
  unsigned char* base = mem.data() + (mis ? cptr::DevArena::kAlign - mis : 0);
  cptr::DevArena a;
  a.init(base, size);
  std::mt19937 rng(7);
  struct Piece { unsigned char* p; size_t n; };
  std::vector<Piece> live;
  std::vector<int> owner(size, -1);
  size_t expect = 0;
  for (int it = 0; it < 20000; ++it) {
    if (live.empty() || rng() % 3) {
      const size_t n = 1 + rng() % 20000;
      void* p = a.alloc(n);
      if (!p) {
        if (a.largest_free() >= cptr::DevArena::round(n)) { std::printf("FAIL: alloc refused\n"); return 1; }
        continue;
      }
      unsigned char* q = static_cast<unsigned char*>(p);
      const size_t off = q - base;
      if (off % cptr::DevArena::kAlign || off + n > size) { std::printf("FAIL: bad piece\n"); return 1; }
      for (size_t i = off; i < off + cptr::DevArena::round(n); ++i) {
        if (owner[i] != -1) { std::printf("FAIL: overlap\n"); return 1; }
        owner[i] = 1;
      }
      live.push_back({q, n});
      expect += cptr::DevArena::round(n);
    } else {
      const size_t k = rng() % live.size();
      const size_t off = live[k].p - base;
      for (size_t i = off; i < off + cptr::DevArena::round(live[k].n); ++i) owner[i] = -1;
      if (!a.release(live[k].p)) { std::printf("FAIL: release refused\n"); return 1; }
      if (a.release(live[k].p)) { std::printf("FAIL: double release accepted\n"); return 1; }
      expect -= cptr::DevArena::round(live[k].n);
      live.erase(live.begin() + k);
    }
    if (a.in_use() != expect) { std::printf("FAIL: in_use\n"); return 1; }
  }
  for (auto& l : live) a.release(l.p);
  if (a.in_use() != 0 || a.largest_free() != size) { std::printf("FAIL: not coalesced\n"); return 1; }
  std::printf("OK\n");
  return 0;
}
