// Host-only unit tests of the runtime's LRU binding/graph cache and the
// tuned-table parser (no HIP).  Prints "ok" and exits 0 on success.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "lru_cache.hpp"
#include "tuning.hpp"

#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                           \
    }                                                         \
  } while (0)

int main() {
  using pcoll::LruCache;
  std::vector<int> disposed;
  {
    LruCache<int, int> c(3, [&](const int& k, int&) { disposed.push_back(k); });
    CHECK(c.get(1) == nullptr);
    c.put(1, 10);
    c.put(2, 20);
    c.put(3, 30);
    CHECK(*c.get(1) == 10);  // 1 becomes most recent; LRU is 2
    c.put(4, 40);            // evicts 2
    CHECK(disposed.size() == 1 && disposed[0] == 2);
    CHECK(c.get(2) == nullptr);
    CHECK(*c.get(3) == 30 && *c.get(4) == 40 && *c.get(1) == 10);
    c.put(5, 50);  // LRU now 3
    CHECK(disposed.back() == 3);
    c.put(1, 11);  // replace disposes the old value, no eviction
    CHECK(disposed.back() == 1 && c.size() == 3 && *c.get(1) == 11);
    CHECK(c.evictions() == 2);
    CHECK(c.hits() == 5 && c.misses() == 2);
  }
  CHECK(disposed.size() == 6);  // clear() at destruction disposes the rest
  {
    LruCache<int, int> c(0, [](const int&, int&) {});
    CHECK(c.capacity() == 1);
    c.put(1, 1);
    c.put(2, 2);
    CHECK(c.size() == 1 && c.get(1) == nullptr && *c.get(2) == 2);
  }
  // tuned table
  const std::string t =
      "# dtype op ranks graph log2_lo log2_hi tile groups_per_cu\n"
      "f32 sum 8 0 24 30 8192 2   # large messages\n"
      "f32 sum * * 0 23 4096 1\n"
      "bf16 * * 1 * * 16384 4\n"
      "garbage line\n"
      "f32 sum 8 0 0 63 1000 2\n"  // tile not a multiple of 1024: skipped
      "i32 max 16 0 0 63 2048 3 1 4 8 4 extra\n"  // 13 fields: skipped
      "i32 max 16 0 0 63 2048 3 1 4 8 3\n"  // unroll 3: skipped
      "i32 max 16 0 0 63 2048 3 1 4 65\n"    // batch 65: skipped
      "i32 max 16 0 0 63 2048 3 1 9\n"        // 9 waves: skipped
      "i32 sum 16 0 0 63 2048 3 -1\n"       // negative interleave: skipped
      "i32 max 16 0 0 63 2048 3 1\n"
      "bf16 max 4 0 0 63 8192 1 1 2 32\n"
      "e4m3 sum 8 1 0 63 32768 2 4 8 64 2\n";
  auto rows = pcoll::parse_tune_table(t);
  CHECK(rows.size() == 6);
  auto c1 = pcoll::tune_lookup(rows, 1, 0, 8, 0, 1ull << 26);
  CHECK(c1.tile_elems == 8192 && c1.groups_per_cu == 2);
  auto c2 = pcoll::tune_lookup(rows, 1, 0, 8, 0, 1ull << 20);
  CHECK(c2.tile_elems == 4096 && c2.groups_per_cu == 1);
  auto c3 = pcoll::tune_lookup(rows, 2, 1, 3, 1, 123);
  CHECK(c3.tile_elems == 16384 && c3.groups_per_cu == 4);
  auto c4 = pcoll::tune_lookup(rows, 0, 0, 16, 0, 1ull << 26);  // default
  CHECK(c4.tile_elems == 4096 && c4.groups_per_cu == 2 && c4.interleave == 0);
  auto c6 = pcoll::tune_lookup(rows, 0, 1, 16, 0, 1ull << 26);
  CHECK(c6.tile_elems == 2048 && c6.groups_per_cu == 3 && c6.interleave == 1 &&
        c6.group_waves == 4 && c6.publish_batch == 16 && c6.unroll == 4);
  auto c8 = pcoll::tune_lookup(rows, 3, 0, 8, 1, 1ull << 30);  // graph row
  CHECK(c8.tile_elems == 32768 && c8.unroll == 2);
  auto c9 = pcoll::tune_lookup(rows, 3, 0, 8, 0, 1ull << 30);  // no row
  CHECK(c9.tile_elems == 16384 && c9.unroll == 4);
  auto c7 = pcoll::tune_lookup(rows, 2, 1, 4, 0, 1ull << 20);
  CHECK(c7.tile_elems == 8192 && c7.group_waves == 2 && c7.publish_batch == 32);
  auto c5 = pcoll::tune_lookup(rows, 1, 0, 8, 0, 1ull << 31);  // beyond 30
  CHECK(c5.tile_elems == 4096);
  std::printf("ok\n");
  return 0;
}
