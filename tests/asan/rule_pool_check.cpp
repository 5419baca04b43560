// Host check of the step rule's thread pool (csrc/rule_pool.hpp), built with the address
// and undefined-behaviour sanitizers or with the thread sanitizer: every part runs once
// per call, a part that throws is rethrown to the caller only after every part has ended,
// the pool stays usable afterwards, and pools are created and destroyed cleanly.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <stdexcept>
#include <vector>

#include "rule_pool.hpp"

#define CHECK(cond)                                              \
  do {                                                           \
    if (!(cond)) {                                               \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      std::exit(1);                                              \
    }                                                            \
  } while (0)

int main() {
  for (int threads = 1; threads <= 16; threads *= 2) {
    tsbts::RulePool pool(threads);
    CHECK(pool.parts() == threads);
    // every part once per call, over many calls; plain writes to per-part slots
    std::vector<long> hits(threads, 0);
    for (int call = 0; call < 2000; ++call) {
      const std::function<void(int, int)> f = [&](int w, int np) {
        CHECK(np == threads && w >= 0 && w < np);
        ++hits[w];
      };
      pool.run(f);
    }
    for (int w = 0; w < threads; ++w) CHECK(hits[w] == 2000);
    // a throwing part (a worker's, then the caller's own): the call rethrows after every
    // other part has finished its work
    for (int bad = 0; bad < threads; ++bad) {
      std::atomic<int> finished{0};
      const std::function<void(int, int)> f = [&](int w, int) {
        if (w == bad) throw std::runtime_error("part failed");
        for (volatile int spin = 0; spin < 20000; ++spin) {
        }
        finished.fetch_add(1);
      };
      bool thrown = false;
      try {
        pool.run(f);
      } catch (const std::runtime_error &) {
        thrown = true;
      }
      CHECK(thrown);
      CHECK(finished.load() == threads - 1);
    }
    // still usable after the failures
    std::atomic<int> count{0};
    const std::function<void(int, int)> g = [&](int, int) { count.fetch_add(1); };
    pool.run(g);
    CHECK(count.load() == threads);
  }
  // pools that never ran a job
  for (int k = 0; k < 50; ++k) tsbts::RulePool idle(1 + k % 8);
  std::printf("rule pool check ok\n");
  return 0;
}
