// Stress of libdc's host thread pool: many short rounds back to back, each
// with its own work function, from two callers on two pools at once. Every
// item of every round must run exactly once with its own round's function.
#include <stdio.h>

#include <atomic>
#include <thread>
#include <vector>

#include "dc_host.h"

// defined beside the kernels in the library; the pool does not use it
namespace dc {
int device_cu_count() { return 256; }
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

int main(int argc, char** argv) {
  const int rounds = argc > 1 ? atoi(argv[1]) : 20000;
  dc::Pool a(8), b(8);
  int bad_a = 0, bad_b = 0;
  std::thread t([&] { bad_b = stress(b, rounds, 5); });
  bad_a = stress(a, rounds, 3);
  t.join();
  printf("rounds %d, bad items %d %d\n", rounds, bad_a, bad_b);
  return bad_a || bad_b;
}
