// Host-only stress check of the streaming pipeline's batch ring and planner:
// loader threads fill slots with random delays, the consumer takes batches in
// order with random delays and releases each slot one batch late, exactly as
// the streaming pass does.  Every batch must arrive once, in order, with its
// own content; a failing fill must stop the pass without a hang.
#include <chrono>
#include <cstdio>
#include <random>
#include <thread>
#include <vector>

#include "ivx_stream_engine.h"

using namespace ivx;

static void nap(std::mt19937& g, int max_us) {
  std::uniform_int_distribution<int> d(0, max_us);
  std::this_thread::sleep_for(std::chrono::microseconds(d(g)));
}

// returns the number of batches the consumer received, or -1 on a mismatch
static long run(int nslots, int nloaders, long nb, long fail_at, unsigned seed) {
  BatchRing ring(nslots, nb);
  std::vector<long> slot_content(nslots, -1);
  std::vector<int> writes(nb, 0);
  auto fill = [&](int64_t b, int s) -> bool {
    thread_local std::mt19937 g(seed * 7919u + (unsigned)std::hash<std::thread::id>()(
                                                   std::this_thread::get_id()));
    nap(g, 200);
    if (b == fail_at) return false;
    slot_content[s] = b;
    writes[b] += 1;
    return true;
  };
  std::vector<std::thread> th;
  for (int i = 0; i < nloaders; ++i) th.emplace_back([&] { ring.loader_loop(fill); });
  std::mt19937 g(seed);
  long got = 0;
  bool bad = false;
  for (long b = 0; b < nb; ++b) {
    if (!ring.wait_ready(b)) break;
    if (slot_content[ring.slot_of(b)] != b) bad = true;
    nap(g, 150);
    ++got;
    if (b >= 1) ring.release(b - 1);
  }
  ring.stop();
  for (auto& t : th) t.join();
  for (long b = 0; b < got; ++b)
    if (writes[b] != 1) bad = true;
  if (fail_at < 0 && got != nb) bad = true;
  if (fail_at >= 0 && got > fail_at) bad = true;
  if (fail_at >= 0 && !ring.failed()) bad = true;
  return bad ? -1 : got;
}

int main() {
  int cases = 0;
  for (int nslots = 2; nslots <= 5; ++nslots)
    for (int nl = 1; nl <= 6; ++nl)
      for (long nb : {0L, 1L, 2L, 3L, 7L, 40L}) {
        for (long fail_at : {-1L, 0L, nb / 2, nb - 1}) {
          if (fail_at >= nb) continue;
          if (run(nslots, nl, nb, fail_at, 1000u + (unsigned)cases) < 0) {
            std::printf("FAIL slots=%d loaders=%d batches=%ld fail_at=%ld\n", nslots, nl, nb,
                        fail_at);
            return 1;
          }
          ++cases;
        }
      }
  // planner: every batch within the limits, consecutive, and maximal
  std::mt19937 g(5);
  for (int it = 0; it < 2000; ++it) {
    const long U = g() % 60;
    const long mu = 1 + g() % 9, mf = 1 + g() % 400;
    std::vector<int64_t> off(U + 1, 0);
    for (long u = 0; u < U; ++u) off[u + 1] = off[u] + (int64_t)(g() % (mf + 1));
    std::vector<int64_t> st;
    const int64_t nb = plan_batches(off.data(), U, mu, mf, st);
    if (nb < 0 || st.front() != 0 || st.back() != U) {
      std::printf("FAIL planner U=%ld\n", U);
      return 1;
    }
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t u0 = st[b], u1 = st[b + 1];
      const bool fits = u1 > u0 && u1 - u0 <= mu && off[u1] - off[u0] <= mf;
      const bool maximal = u1 == U || u1 - u0 == mu || off[u1 + 1] - off[u0] > mf;
      if (!fits || !maximal) {
        std::printf("FAIL planner batch %ld\n", (long)b);
        return 1;
      }
    }
  }
  std::printf("OK %d ring cases\n", cases);
  return 0;
}
