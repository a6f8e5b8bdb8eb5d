// Sanitizer driver (test infrastructure): exercises the host C/C++ code of this
// repository -- the oracle (oracle/lob_oracle.c), the workload generator
// (paper_2308_13289_amd/workload/flowgen.c) and the replay-window cutter
// (paper_2308_13289_amd/csrc/lob_windows.cpp) -- on inputs that reach their edges,
// for a build with AddressSanitizer and UndefinedBehaviorSanitizer.  Exits 0 when
// every call returned what it should; the sanitizers abort on the first finding.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "flowgen.h"
#include "lob.h"
#include "lob_oracle.h"

namespace {

int failures = 0;

void check(bool ok, const char *what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

// splitmix64: the driver's own input stream
uint64_t mix(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int32_t pick(uint64_t &s, const std::vector<int32_t> &v) { return v[mix(s) % v.size()]; }

// One book, random messages with quantities up to INT32_MAX, repeated and
// decreasing times, cancels of live, unknown and initial orders, a full side.
void oracle_edges() {
  uint64_t s = 7;
  const std::vector<int32_t> qty = {0, -3, 1, 2, 3, 1 << 24, 1000000000, 2000000000, INT32_MAX};
  for (int32_t cap : {1, 2, 3, 64, 130}) {
    orc_book *b = orc_new(cap);
    check(b != nullptr, "orc_new");
    // start from an L2 snapshot: asks 103, 104; bids 101, 100 (one refused first)
    const int32_t bad[2 * 2 * 2] = {103, 5, 102, 5, 101, 5, 100, 5};  // asks not ascending
    check(orc_seed_l2(b, bad, 2, 0, 1, 0) < 0, "seed refuses a snapshot that is not a book");
    const int32_t good[2 * 2 * 2] = {103, INT32_MAX, 104, 7, 101, INT32_MAX, 100, 9};
    const int32_t placed = orc_seed_l2(b, good, 2, 0, 1, 0);
    check(placed == (cap >= 2 ? 4 : -1), "seed places one order per level");
    std::vector<int32_t> trades(8 * (size_t)cap + 8), l2(2 * 10 * 2), dump(6 * (size_t)cap);
    for (int k = 0; k < 4000; ++k) {
      int32_t m[8];
      m[0] = pick(s, {0, 1, 1, 1, 2, 3, 4, 5});
      m[1] = pick(s, {1, -1, 1, -1, 0});
      m[2] = pick(s, {0, 99, 100, 101, 102, 103, 104, 105});
      m[3] = pick(s, qty);
      m[4] = pick(s, {1, 2, 3, 5, 8, -9000, -9001, -9002, -9003, 77});
      m[5] = pick(s, {-1, 0, 4});
      m[6] = pick(s, {0, 1, 2});
      m[7] = pick(s, {0, 1, 999999999});
      const int32_t n = orc_process(b, m, trades.data(), cap + 1);
      check(n >= 0 && n <= cap + 1, "trades of one message fit the bound");
      if (k % 97 == 0) {
        orc_l2(b, 10, l2.data());
        check(orc_dump(b, k & 1, dump.data()) >= 0, "dump");
      }
    }
    orc_stats st;
    orc_get_stats(b, &st);
    check(st.n_msgs == 4000, "message count");
    orc_free(b);
  }
}

// The generator's ragged, uniform, agent and request streams at small sizes, and
// the oracle's batch runner over them on several threads.
void generator_and_batch() {
  const int32_t n = 96;
  std::vector<int32_t> caps(n), mids(n), seeds(n);
  std::vector<int64_t> flow(n), offs(n + 1, 0);
  fg_ragged_params(230813289ull, 2, n, caps.data(), flow.data(), mids.data());
  for (int32_t i = 0; i < n; ++i) {
    check(caps[i] == 50 || caps[i] == 100 || caps[i] == 500 || caps[i] == 1000, "ragged capacity");
    flow[i] = flow[i] > 3000 ? 3000 : flow[i];
    seeds[i] = caps[i] / 2;
    offs[i + 1] = offs[i] + 2 * seeds[i] + flow[i];
  }
  std::vector<int32_t> msgs(8 * (size_t)offs[n]);
  check(fg_generate(230813289ull, 2, n, nullptr, mids.data(), 100, caps.data(), seeds.data(), flow.data(),
                    msgs.data(), offs.data(), 4) == 0,
        "fg_generate");
  const int32_t steps = 5;
  std::vector<int32_t> times(2 * (size_t)n * steps, 34200), acts((size_t)n * steps * 4 * 8);
  check(fg_agent(230813289ull, 3, n, nullptr, mids.data(), 100, steps, times.data(), acts.data(), 2) == 0,
        "fg_agent");
  std::vector<int64_t> arrival(500);
  std::vector<int32_t> book(500), kind(500), size(500);
  fg_requests(230813289ull, 4, 500, 200000.0, n, arrival.data(), book.data(), kind.data(), size.data());
  for (int k = 1; k < 500; ++k) check(arrival[k] >= arrival[k - 1], "arrivals in order");
  // the oracle over every book, per-message L2, dumps, on 4 threads
  std::vector<int64_t> toffs(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) toffs[i + 1] = toffs[i] + 2 * (offs[i + 1] - offs[i]) + caps[i];
  std::vector<int32_t> trades(8 * (size_t)toffs[n]), l2((size_t)offs[n] * 2 * 3 * 2), dumps((size_t)n * 2 * 1000 * 6);
  std::vector<int64_t> tmsg(toffs[n]), counts(n);
  std::vector<orc_stats> stats(n);
  check(orc_run(n, caps.data(), msgs.data(), offs.data(), ORC_L2_PER_MESSAGE, 3, l2.data(), trades.data(),
                toffs.data(), tmsg.data(), counts.data(), stats.data(), dumps.data(), 1000, 4) == 0,
        "orc_run");
  for (int32_t i = 0; i < n; ++i) check(counts[i] <= toffs[i + 1] - toffs[i], "trade room");
  // windows of book 0's stream
  const int64_t m0 = offs[1];
  std::vector<int32_t> win((size_t)3 * 40 * 16 * 8), wsteps(3);
  std::vector<int64_t> first(4);
  const lob_status ws = lob_windows(msgs.data(), m0, 34200, 1, 16, 40, 3, win.data(), wsteps.data(), first.data());
  check(ws == LOB_OK || ws == LOB_ECAP, "lob_windows");
  check(lob_windows(msgs.data(), m0, 34200, 1, 16, 40, 3, nullptr, wsteps.data(), first.data()) != LOB_EINVAL,
        "lob_windows counting");
  check(lob_windows(msgs.data(), m0, 34200, 0, 16, 40, 3, nullptr, wsteps.data(), first.data()) == LOB_EINVAL,
        "lob_windows refuses a window of 0 s");
}

}  // namespace

int main() {
  oracle_edges();
  generator_and_batch();
  if (failures) return 1;
  std::puts("sanitize driver ok");
  return 0;
}
