// Randomised check of the batch workspace allocator: blocks never overlap,
// stay inside the range and 256-byte aligned, and freeing everything gives
// back one block of the full size.  Built and run by test_host_logic.py.
#include <cassert>
#include <cstdio>
#include <random>

#include "arena.h"

int main() {
  using lbm_host::Arena;
  std::mt19937 rng(1);
  for (int trial = 0; trial < 300; ++trial) {
    Arena a;
    const size_t N = size_t(1) << 20;
    a.reset(N);
    std::map<size_t, size_t> live;  // offset -> bytes
    for (int op = 0; op < 400; ++op) {
      if (live.empty() || rng() % 3) {
        const size_t bytes = rng() % 40000 + 1;
        size_t off = 0;
        const bool top = rng() % 4 == 0;
        if (!(top ? a.alloc_top(bytes, &off) : a.alloc(bytes, &off))) continue;
        const size_t b = lbm_host::arena_align(bytes);
        if (off % 256 || off + b > N) return 1;
        for (const auto &kv : live)
          if (!(off + b <= kv.first || kv.first + kv.second <= off)) return 2;
        live[off] = b;
      } else {
        auto it = live.begin();
        std::advance(it, rng() % live.size());
        a.release(it->first, it->second);
        live.erase(it);
      }
    }
    for (const auto &kv : live) a.release(kv.first, kv.second);
    if (a.largest() != N) return 3;
  }
  std::puts("arena ok");
  return 0;
}
