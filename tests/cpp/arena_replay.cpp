// Replays the device builds of solve-server requests through DevArena.
//
// Input (stdin): the allocation plan of one request's device build, as
// cptr_export(CPTR_EXPORT_DEVICE_PLAN) gives it (n, then n entries: bytes > 0
// allocates, -1 - k releases the k-th allocation), then N (DOF), the budget
// as a multiple of the request's footprint, the number of requests, the
// number admitted at a time, and the number of random schedules.
//
// Each request, once admitted, runs its plan, then takes its right-hand side
// and solution (two vectors of N doubles), then releases everything (the end
// of its solve).  Requests admitted together advance one step at a time in a
// random order, like the slot threads of the server.  A step whose
// allocation finds no contiguous piece is a failed build: the request
// releases all it holds (the path of a failed setup_device) and is admitted
// again later.  The program prints the number of schedules that saw at least
// one failed build, the number of failed builds, and checks the arena's
// bookkeeping throughout (no overlap, everything returned at the end).
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "dev_arena.hpp"

int main() {
  long n = 0;
  if (std::scanf("%ld", &n) != 1) return 2;
  std::vector<int64_t> plan((size_t)n);
  for (long i = 0; i < n; ++i)
    if (std::scanf("%ld", &plan[(size_t)i]) != 1) return 2;
  long ndof = 0, nreq = 0, together = 0, schedules = 0;
  double mult = 0;
  if (std::scanf("%ld %lf %ld %ld %ld", &ndof, &mult, &nreq, &together, &schedules) != 5) return 2;
  const int64_t vec = (int64_t)cptr::DevArena::round(sizeof(double) * (size_t)ndof);
  int64_t footprint = 2 * vec;
  for (int64_t v : plan)
    if (v > 0) footprint += v;
  const size_t size = (size_t)((double)footprint * mult) / cptr::DevArena::kAlign * cptr::DevArena::kAlign;
  // a host region stands in for the device arena (never touched)
  std::vector<unsigned char> mem(size + cptr::DevArena::kAlign);
  unsigned char* base = mem.data();
  base += (cptr::DevArena::kAlign - reinterpret_cast<uintptr_t>(base) % cptr::DevArena::kAlign) % cptr::DevArena::kAlign;
  std::mt19937_64 rng(11892);
  long bad_schedules = 0, failed_builds = 0;
  for (long sc = 0; sc < schedules; ++sc) {
    cptr::DevArena a;
    a.init(base, size);
    struct Run { size_t step = 0; std::vector<void*> held; std::vector<void*> byidx; };
    std::vector<Run> slots;
    long next = 0, done = 0, fails = 0;
    auto release_all = [&](Run& r) {
      for (void* p : r.held)
        if (p && !a.release(p)) { std::printf("FAIL: release refused\n"); std::exit(1); }
      r.held.clear();
      r.byidx.clear();
    };
    std::vector<long> queue;
    for (long q = 0; q < nreq; ++q) queue.push_back(q);
    while (done < nreq) {
      while ((long)slots.size() < together && next < (long)queue.size()) {
        slots.emplace_back();
        ++next;
      }
      const size_t k = rng() % slots.size();
      Run& r = slots[k];
      const size_t total = plan.size() + 2;
      if (r.step < total) {
        const int64_t v = r.step < plan.size() ? plan[r.step] : vec;
        if (v > 0) {
          void* p = a.alloc((size_t)v);
          if (!p) {  // failed build: everything back, tried again later
            ++fails;
            release_all(r);
            r.step = 0;
            queue.push_back(-1);
            slots.erase(slots.begin() + (long)k);
            continue;
          }
          r.held.push_back(p);
          r.byidx.push_back(p);
        } else {
          const size_t idx = (size_t)(-1 - v);
          void* p = r.byidx.at(idx);
          for (auto& h : r.held)
            if (h == p) h = nullptr;
          if (!a.release(p)) { std::printf("FAIL: release refused\n"); return 1; }
        }
        ++r.step;
      } else {  // solve done: everything back
        release_all(r);
        slots.erase(slots.begin() + (long)k);
        ++done;
      }
    }
    if (a.in_use() != 0 || a.largest_free() != a.size()) { std::printf("FAIL: arena not empty\n"); return 1; }
    if (fails) ++bad_schedules;
    failed_builds += fails;
  }
  std::printf("schedules %ld with_failed_build %ld failed_builds %ld footprint %ld arena %zu\n", schedules,
              bad_schedules, failed_builds, (long)footprint, size);
  return 0;
}
