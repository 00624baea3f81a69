// Host check of the request server's arena allocator: random allocations
// and releases against a byte map of the arena.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "gmunu_pool.hpp"

#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      std::printf("FAIL %s line %d\n", #c, __LINE__);         \
      std::exit(1);                                           \
    }                                                         \
  } while (0)

int main() {
  const size_t align = 256, cap = 1 << 20;
  gm::RangePool pool(cap + 100, align);
  CHECK(pool.capacity() == cap);
  std::vector<unsigned char> owner(cap / align, 0);
  struct Live {
    size_t off, bytes;
  };
  std::vector<Live> live;
  std::mt19937_64 rng(7);
  for (int it = 0; it < 200000; it++) {
    const bool do_alloc = live.empty() || (rng() % 100) < 55;
    if (do_alloc) {
      const size_t bytes = 1 + rng() % 20000;
      const size_t off = pool.alloc(bytes);
      if (off == gm::RangePool::npos) {
        CHECK(pool.largest_free() < gm::RangePool::round_up(bytes, align));
        continue;
      }
      CHECK(off % align == 0);
      CHECK(off + bytes <= cap);
      for (size_t b = off / align; b < (off + bytes + align - 1) / align; b++) {
        CHECK(owner[b] == 0);
        owner[b] = 1;
      }
      live.push_back({off, bytes});
    } else {
      const size_t k = rng() % live.size();
      const Live l = live[k];
      live[k] = live.back();
      live.pop_back();
      pool.release(l.off, l.bytes);
      for (size_t b = l.off / align; b < (l.off + l.bytes + align - 1) / align; b++) owner[b] = 0;
    }
    size_t used = 0;
    for (auto &l : live) used += gm::RangePool::round_up(l.bytes, align);
    CHECK(pool.used() == used);
    CHECK(pool.peak() >= used);
  }
  for (auto &l : live) pool.release(l.off, l.bytes);
  CHECK(pool.used() == 0);
  CHECK(pool.fragments() == 1);
  CHECK(pool.largest_free() == cap);
  std::printf("ok\n");
  return 0;
}
