// Randomised check of the serving arena against a byte-map model: ranges
// handed out never overlap and lie inside the arena, a request fails only when
// no free range is large enough, alloc takes the lowest fitting range, and
// after everything is returned the arena is one free range again.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "zg_arena.h"

int main(int argc, char **argv) {
  const uint64_t size = 1 << 16;
  const int steps = argc > 1 ? std::atoi(argv[1]) : 200000;
  std::mt19937_64 rng(12345);
  zg::Arena a;
  a.init(size);
  std::vector<uint8_t> used(size, 0);
  struct Live { uint64_t off, bytes; };
  std::vector<Live> live;
  for (int step = 0; step < steps; ++step) {
    const bool do_alloc = live.empty() || (rng() % 100) < 55;
    if (do_alloc) {
      const uint64_t bytes = 1 + rng() % (rng() % 8 == 0 ? 8192 : 512);
      // the lowest offset with `bytes` free bytes in the model
      uint64_t want = UINT64_MAX, run = 0;
      for (uint64_t i = 0; i < size; ++i) {
        run = used[i] ? 0 : run + 1;
        if (run == bytes) { want = i + 1 - bytes; break; }
      }
      uint64_t off = 0;
      const bool ok = a.alloc(bytes, &off);
      if (ok != (want != UINT64_MAX)) { std::printf("FAIL step %d: alloc %d, model %d\n", step, ok, want != UINT64_MAX); return 1; }
      if (!ok) continue;
      if (off != want) { std::printf("FAIL step %d: first fit %llu, model %llu\n", step, (unsigned long long)off, (unsigned long long)want); return 1; }
      if (off + bytes > size) { std::printf("FAIL step %d: out of range\n", step); return 1; }
      for (uint64_t i = off; i < off + bytes; ++i) {
        if (used[i]) { std::printf("FAIL step %d: overlap at %llu\n", step, (unsigned long long)i); return 1; }
        used[i] = 1;
      }
      live.push_back({off, bytes});
    } else {
      const size_t k = rng() % live.size();
      const Live l = live[k];
      live[k] = live.back();
      live.pop_back();
      a.release(l.off, l.bytes);
      for (uint64_t i = l.off; i < l.off + l.bytes; ++i) used[i] = 0;
    }
    // free ranges are disjoint, sorted, coalesced and agree with the model
    uint64_t prev_end = 0, free_bytes = 0;
    bool first = true;
    for (const auto &r : a.free_ranges()) {
      if (!first && r.first <= prev_end) { std::printf("FAIL step %d: ranges not coalesced\n", step); return 1; }
      for (uint64_t i = r.first; i < r.first + r.second; ++i)
        if (used[i]) { std::printf("FAIL step %d: free range over used byte\n", step); return 1; }
      prev_end = r.first + r.second;
      free_bytes += r.second;
      first = false;
    }
    uint64_t model_free = 0;
    for (uint64_t i = 0; i < size; ++i) model_free += !used[i];
    if (free_bytes != model_free) { std::printf("FAIL step %d: free bytes %llu, model %llu\n", step, (unsigned long long)free_bytes, (unsigned long long)model_free); return 1; }
  }
  for (const Live &l : live) a.release(l.off, l.bytes);
  if (a.free_ranges().size() != 1 || a.free_ranges().begin()->second != size) { std::printf("FAIL: not one range at the end\n"); return 1; }
  std::printf("ok %d steps\n", steps);
  return 0;
}
