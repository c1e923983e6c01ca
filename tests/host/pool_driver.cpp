// Driver of the thread-pool test (tests/test_host_pool_tsan.py): the test splices the
// pool and parallel loop of msdd.cpp in at the marker below and builds this file with
// ThreadSanitizer on the CPU.
#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>
#include <cstdio>
#include <cstdint>
#include <string>
struct MsddError { int code; std::string msg; };
// @@POOL@@
int main() {
  long total = 0;
  for (int rep = 0; rep < 2000; ++rep) {
    const int n = 1 + rep % 300, nthr = 1 + rep % 16;
    std::vector<int> hit(n, 0);
    parallel_for(n, nthr, [&](int i, int t) { hit[i] += 1 + (t >= 0 ? 0 : 1); });
    for (int i = 0; i < n; ++i) if (hit[i] != 1) { std::printf("bad %d %d\n", rep, i); return 1; }
    total += n;
  }
  // errors propagate
  bool caught = false;
  try { parallel_for(100, 8, [&](int i, int) { if (i == 37) throw MsddError{5, "x"}; }); }
  catch (const MsddError& e) { caught = e.code == 5; }
  if (!caught) { std::printf("no error\n"); return 1; }
  // two caller threads at once (one gets the pool, the other its own threads)
  std::atomic<long> sum(0);
  std::thread a([&] { for (int r = 0; r < 200; ++r) parallel_for(500, 16, [&](int i, int) { sum += i; }); });
  std::thread b([&] { for (int r = 0; r < 200; ++r) parallel_for(500, 16, [&](int i, int) { sum += i; }); });
  a.join(); b.join();
  if (sum != 2L * 200 * (499L * 500 / 2)) { std::printf("bad sum\n"); return 1; }
  std::printf("ok %ld\n", total);
  return 0;
}
