// Host-only test of the server's pool allocator when host memory runs out:
// global operator new is replaced by one that throws std::bad_alloc on a
// chosen call, and random alloc/release sequences check that a throwing
// operation leaves the allocator exactly as it was (its free list and byte
// count), while the operations that succeed keep matching a byte-map model.
// Built with g++ under AddressSanitizer by test_pool_allocator.py.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <new>
#include <random>
#include <vector>

#include "syev3_pool.hpp"

static long g_fail_in = -1;  // throw on the g_fail_in-th allocation from now (0 = next)
static long g_throws = 0;

void* operator new(std::size_t n) {
  if (g_fail_in >= 0 && g_fail_in-- == 0) {
    ++g_throws;
    throw std::bad_alloc();
  }
  if (void* p = std::malloc(n ? n : 1)) return p;
  throw std::bad_alloc();
}
void operator delete(void* p) noexcept { std::free(p); }
void operator delete(void* p, std::size_t) noexcept { std::free(p); }

int main() {
  const size_t size = 1 << 16;
  syev3::PoolAllocator pool(size);
  std::vector<unsigned char> used(size, 0);
  struct Block { size_t off, len; };
  std::vector<Block> live;
  live.reserve(1 << 12);
  std::mt19937_64 rng(777);
  size_t in_use = 0;
  long failed_ops = 0;
  for (int step = 0; step < 40000; ++step) {
    const std::map<size_t, size_t> before = pool.free_ranges();
    const size_t in_use_before = pool.in_use();
    g_fail_in = (rng() % 2) ? 0 : -1;  // half the operations meet an exhausted heap
    bool threw = false;
    if (live.empty() || rng() % 3 != 0) {
      const size_t len = 256 * (1 + rng() % 16);
      size_t off = 0;
      bool ok = false;
      try {
        ok = pool.alloc(len, &off);
      } catch (const std::bad_alloc&) {
        threw = true;
      }
      g_fail_in = -1;
      if (!threw && ok) {
        for (size_t k = off; k < off + len; ++k) {
          if (used[k]) { std::printf("overlap at %zu\n", k); return 1; }
          used[k] = 1;
        }
        live.push_back({off, len});
        in_use += len;
      }
    } else {
      const size_t i = rng() % live.size();
      try {
        pool.release(live[i].off, live[i].len);
      } catch (const std::bad_alloc&) {
        threw = true;
      }
      g_fail_in = -1;
      if (!threw) {
        for (size_t k = live[i].off; k < live[i].off + live[i].len; ++k) used[k] = 0;
        in_use -= live[i].len;
        live[i] = live.back();
        live.pop_back();
      }
    }
    if (threw) {
      ++failed_ops;
      if (pool.free_ranges() != before || pool.in_use() != in_use_before) {
        std::printf("step %d: a throwing operation changed the allocator\n", step);
        return 1;
      }
    }
    if (pool.in_use() != in_use) { std::printf("in_use mismatch at step %d\n", step); return 1; }
    // the free list is exactly the model's free runs, coalesced
    size_t k = 0;
    std::map<size_t, size_t> runs;
    while (k < size) {
      if (used[k]) { ++k; continue; }
      size_t j = k;
      while (j < size && !used[j]) ++j;
      runs[k] = j - k;
      k = j;
    }
    if (runs != pool.free_ranges()) { std::printf("free list differs at step %d\n", step); return 1; }
  }
  if (failed_ops < 1000 || g_throws != failed_ops) {
    std::printf("too few injected failures: %ld (throws %ld)\n", failed_ops, g_throws);
    return 1;
  }
  for (auto& b : live) pool.release(b.off, b.len);
  size_t off;
  if (pool.in_use() != 0 || !pool.alloc(size, &off) || off != 0) {
    std::printf("pool not whole after releasing everything\n");
    return 1;
  }
  std::printf("pool exception-safe: %ld operations met a failing allocation\n", failed_ops);
  return 0;
}
