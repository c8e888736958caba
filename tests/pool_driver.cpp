// Host-only randomized test of the server's pool allocator against a
// reference model (a byte map), built with g++ by test_pool_allocator.py.
#include <cstdio>
#include <random>
#include <vector>

#include "syev3_pool.hpp"

int main() {
  const size_t size = 1 << 16;
  syev3::PoolAllocator pool(size);
  std::vector<unsigned char> used(size, 0);
  struct Block { size_t off, len; };
  std::vector<Block> live;
  std::mt19937_64 rng(12345);
  size_t in_use = 0;
  for (int step = 0; step < 60000; ++step) {
    if (live.empty() || rng() % 3 != 0) {
      const size_t len = 256 * (1 + rng() % 16);
      size_t off;
      if (pool.alloc(len, &off)) {
        if (off + len > size) { std::printf("out of range\n"); return 1; }
        for (size_t k = off; k < off + len; ++k) {
          if (used[k]) { std::printf("overlap at %zu\n", k); return 1; }
          used[k] = 1;
        }
        live.push_back({off, len});
        in_use += len;
      } else {
        // first fit must have failed for real: no free run of len bytes
        size_t run = 0, best = 0;
        for (size_t k = 0; k < size; ++k) { run = used[k] ? 0 : run + 1; if (run > best) best = run; }
        if (best >= len) { std::printf("missed a free run of %zu >= %zu\n", best, len); return 1; }
      }
    } else {
      const size_t i = rng() % live.size();
      pool.release(live[i].off, live[i].len);
      for (size_t k = live[i].off; k < live[i].off + live[i].len; ++k) used[k] = 0;
      in_use -= live[i].len;
      live[i] = live.back();
      live.pop_back();
    }
    if (pool.in_use() != in_use) { std::printf("in_use mismatch\n"); return 1; }
  }
  for (auto& b : live) pool.release(b.off, b.len);
  size_t off;
  if (pool.in_use() != 0 || !pool.alloc(size, &off) || off != 0) {
    std::printf("pool not whole after releasing everything\n");
    return 1;
  }
  std::printf("pool ok\n");
  return 0;
}
