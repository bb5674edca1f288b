// Host-only check of the device-arena sub-allocator (first-fit ranges with an
// exact-size cache in front, and last-fit short-lived blocks released straight
// to the range map).  Seeded random allocate/release sequences, a third of
// them short-lived, over a 64 MiB arena of offsets (the base is never
// dereferenced); the invariants:
// every range is aligned and inside the arena, live ranges never overlap,
// used() is the sum of the live sizes, a request is refused only when no
// aligned gap of its size exists between the live ranges, and releasing
// everything leaves one free range of the whole arena.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "internal.h"

namespace {

struct Live {
  size_t off, bytes, align;
  bool high;
};

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

int main(int argc, char** argv) {
  const unsigned seed = argc > 1 ? unsigned(std::atoi(argv[1])) : 1u;
  const int steps = argc > 2 ? std::atoi(argv[2]) : 200000;
  std::mt19937_64 rng(seed);
  const size_t size = size_t(64) << 20;
  spamm::Arena arena;
  arena.init(nullptr, size);
  std::vector<Live> live;
  size_t allocs = 0, refused = 0, releases = 0;

  auto invariants = [&]() -> bool {
    std::map<size_t, size_t> m;
    size_t sum = 0;
    for (const Live& l : live) {
      if (l.off % l.align || l.off + l.bytes > size || !m.emplace(l.off, l.bytes).second) return false;
      sum += l.bytes;
    }
    size_t end = 0;
    for (const auto& kv : m) {
      if (kv.first < end) return false;
      end = kv.first + kv.second;
    }
    return sum == arena.used();
  };
  auto gap_fits = [&](size_t bytes, size_t align) -> bool {
    std::map<size_t, size_t> m;
    for (const Live& l : live) m[l.off] = l.bytes;
    auto fits = [&](size_t lo, size_t hi) { return round_up(lo, align) + bytes <= hi; };
    size_t cur = 0;
    for (const auto& kv : m) {
      if (kv.first > cur && fits(cur, kv.first)) return true;
      cur = kv.first + kv.second > cur ? kv.first + kv.second : cur;
    }
    return fits(cur, size);
  };

  {  // placement: long-lived from the bottom, short-lived from the top
    const size_t lo = arena.alloc(size_t(1) << 20, 4096), hi = arena.alloc(size_t(1) << 20, 4096, true);
    if (lo != 0 || hi != size - (size_t(1) << 20)) {
      std::printf("FAIL seed %u: placement low %zu high %zu\n", seed, lo, hi);
      return 1;
    }
    arena.release(hi, size_t(1) << 20, 4096, true);
    arena.release(lo, size_t(1) << 20, 4096);
    if (arena.used() != 0 || arena.largest_free() != size) {
      std::printf("FAIL seed %u: placement blocks not returned\n", seed);
      return 1;
    }
  }
  const size_t aligns[] = {256, 512, 4096, 16384, 65536};
  for (int step = 0; step < steps; ++step) {
    if (live.empty() || rng() % 100 < 55) {
      const size_t align = aligns[rng() % 5];
      // repeated power-of-two shapes (exact-size cache hits) and arbitrary sizes
      const size_t bytes = rng() % 4 == 0 ? size_t(1) << (8 + rng() % 14) : 1 + rng() % (size_t(1) << 20);
      const size_t rounded = round_up(bytes, align);
      const bool high = rng() % 3 == 0;
      const size_t off = arena.alloc(bytes, align, high);
      if (off == SIZE_MAX) {
        ++refused;
        if (gap_fits(rounded, align)) {
          std::printf("FAIL seed %u step %d: refused %zu bytes (align %zu) that fit\n", seed, step, rounded, align);
          return 1;
        }
      } else {
        ++allocs;
        live.push_back({off, rounded, align, high});
      }
    } else {
      const size_t i = rng() % live.size();
      arena.release(live[i].off, live[i].bytes, live[i].align, live[i].high);
      live[i] = live.back();
      live.pop_back();
      ++releases;
    }
    if (step % 997 == 0 && !invariants()) {
      std::printf("FAIL seed %u step %d: invariant broken\n", seed, step);
      return 1;
    }
  }
  if (!invariants()) {
    std::printf("FAIL seed %u: invariant broken at the end\n", seed);
    return 1;
  }
  for (const Live& l : live) arena.release(l.off, l.bytes, l.align, l.high);
  live.clear();
  if (arena.used() != 0 || arena.largest_free() != size) {
    std::printf("FAIL seed %u: used %zu, largest free %zu of %zu after releasing everything\n", seed, arena.used(),
                arena.largest_free(), size);
    return 1;
  }
  std::printf("ok seed %u: %zu allocations, %zu refused, %zu releases\n", seed, allocs, refused, releases);
  return 0;
}
