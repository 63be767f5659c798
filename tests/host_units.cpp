// Host-side units of libdc run on the CPU:
//  * the thread pool: many short rounds back to back, each with its own work
//    function, from two callers on two pools at once; every item of every
//    round must run exactly once with its own round's function;
//  * the non-temporal bulk copy: every size and alignment, no byte outside;
//  * the chunk schedule of staged transfers, with and without the ramps at
//    either end: chunks tile [lo, hi) exactly, none is empty or larger than
//    the ring's chunk, for sizes from 0 bytes to 1 TiB (a schedule that
//    doubled past 2^64 once looped forever).
#include <stdio.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

#include "dc_host.h"

// defined beside the kernels in the library; the pool does not use them
namespace dc {
int device_cu_count() { return 256; }
dc_status noalloc_setup(int) { return DC_OK; }
}

static int stress(dc::Pool& pool, int rounds, int salt) {
  int bad = 0;
  for (int r = 0; r < rounds; r++) {
    const int n = 2 + (r * 7 + salt) % 15;
    std::vector<std::atomic<int>> hits(n);
    for (auto& h : hits) h.store(0);
    const int tag = r ^ salt;
    std::atomic<int> wrong{0};
    pool.run(n, [&, tag](int i) {
      if (i < 0 || i >= n || tag != (r ^ salt)) wrong++;
      else hits[i]++;
    });
    for (auto& h : hits) bad += h.load() != 1;
    bad += wrong.load();
  }
  return bad;
}

static int check_bounds() {
  int bad = 0;
  const uint64_t sizes[] = {0, 1, 100, (1ull << 20) - 1, 1ull << 20, (1ull << 20) + 1, 5ull << 20, 128ull << 20,
                            (128ull << 20) + 12345, 958621952ull, 12169061120ull, 1ull << 40};
  for (int ramps = 0; ramps < 4; ramps++)
    for (uint64_t chunk : {1ull << 20, 16ull << 20, 64ull << 20})
      for (uint64_t lo : {0ull, 4096ull, 123456789ull})
        for (uint64_t sz : sizes) {
          const bool up = ramps & 1, down = ramps & 2;
          const std::vector<uint64_t> b = dc::chunk_bounds(lo, lo + sz, chunk, up, down);
          if (b.front() != lo || b.back() != lo + sz) bad++;
          for (size_t i = 0; i + 1 < b.size(); i++)
            if (b[i + 1] <= b[i] || b[i + 1] - b[i] > chunk) bad++;
          if (sz >= (64ull << 20) && b.size() > sz / chunk + 32) bad++;  // full chunks in the middle
          // without a ramp at an end, the chunk there is full (the last one
          // may be the rest)
          if (sz >= 4 * chunk && !up && b[1] - b[0] != chunk) bad++;
          if (sz >= 4 * chunk && !down && b[b.size() - 2] - b[b.size() - 3] != chunk) bad++;
        }
  printf("chunk schedule: %d bad\n", bad);
  return bad;
}

static int check_copy() {
  // non-temporal bulk copy: every size and alignment lands byte for byte
  int bad = 0;
  std::vector<uint8_t> src((2 << 20) + 256), dst((2 << 20) + 256);
  for (size_t i = 0; i < src.size(); i++) src[i] = (uint8_t)(i * 131 + 7);
  const uint64_t sizes[] = {0, 1, 15, 4095, 4096, 4097, 4096 + 63, 65536 + 5, (1u << 20) + 17, 2u << 20};
  for (uint64_t n : sizes)
    for (int so : {0, 1, 8, 15})
      for (int dof : {0, 3, 8, 16, 33}) {
        std::fill(dst.begin(), dst.end(), 0xEE);
        dc::copy_stream(dst.data() + dof, src.data() + so, n);
        for (uint64_t i = 0; i < n; i++) bad += dst[dof + i] != src[so + i];
        bad += dof > 0 && dst[dof - 1] != 0xEE;
        bad += dst[dof + n] != 0xEE;
      }
  printf("bulk copy: %d bad\n", bad);
  return bad;
}

int main(int argc, char** argv) {
  if (check_bounds()) return 2;
  if (check_copy()) return 3;
  const int rounds = argc > 1 ? atoi(argv[1]) : 20000;
  dc::Pool a(8), b(8);
  int bad_a = 0, bad_b = 0;
  std::thread t([&] { bad_b = stress(b, rounds, 5); });
  bad_a = stress(a, rounds, 3);
  t.join();
  printf("rounds %d, bad items %d %d\n", rounds, bad_a, bad_b);
  return bad_a || bad_b;
}
