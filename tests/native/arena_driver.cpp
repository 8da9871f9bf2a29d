// Randomized alloc/release on the server's first-fit arena against a
// brute-force model (one flag per unit), built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitized.py.  Checks: regions
// never overlap or leave the arena, each alloc takes the lowest offset where
// the request fits (first fit) and fails only when no gap fits, used() is the
// sum of live regions, and freeing everything leaves one region.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "server_arena.hpp"

int main() {
  int fails = 0;
  std::mt19937_64 rng(12345);
  long ops = 0;
  for (int trial = 0; trial < 200; ++trial) {
    const size_t size = 1 + rng() % 4096;
    tn::Arena a(size);
    std::vector<char> used(size, 0);
    std::map<size_t, size_t> live;   // off -> n
    size_t live_bytes = 0;
    for (int step = 0; step < 400; ++step, ++ops) {
      const bool do_alloc = live.empty() || rng() % 3 != 0;
      if (do_alloc) {
        const size_t n = 1 + rng() % (size / 4 + 1);
        // model: lowest offset with n free units
        size_t want = size, run = 0;
        for (size_t i = 0; i < size; ++i) {
          run = used[i] ? 0 : run + 1;
          if (run == n) { want = i + 1 - n; break; }
        }
        size_t off = 0;
        const bool ok = a.alloc(n, &off);
        if (ok != (want < size)) { std::fprintf(stderr, "fit mismatch\n"); ++fails; continue; }
        if (!ok) continue;
        if (off != want) { std::fprintf(stderr, "not first fit %zu vs %zu\n", off, want); ++fails; }
        if (off + n > size) { std::fprintf(stderr, "out of arena\n"); ++fails; continue; }
        for (size_t i = off; i < off + n; ++i) {
          if (used[i]) { std::fprintf(stderr, "overlap\n"); ++fails; break; }
          used[i] = 1;
        }
        live[off] = n;
        live_bytes += n;
      } else {
        auto it = live.begin();
        std::advance(it, rng() % live.size());
        a.release(it->first, it->second);
        for (size_t i = it->first; i < it->first + it->second; ++i) used[i] = 0;
        live_bytes -= it->second;
        live.erase(it);
      }
      if (a.used() != live_bytes) { std::fprintf(stderr, "used mismatch\n"); ++fails; }
    }
    for (auto& kv : live) a.release(kv.first, kv.second);
    if (a.used() != 0 || a.free_regions().size() != 1 || a.free_regions().begin()->second != size) {
      std::fprintf(stderr, "not coalesced\n");
      ++fails;
    }
  }
  std::printf("ops %ld fails %d\n", ops, fails);
  return fails ? 1 : 0;
}
