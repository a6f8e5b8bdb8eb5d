// lob_windows.cpp -- windowed replay data (JAX-LOB Section 5.1.1, data loading).
//
// Host code only: one book's message stream is cut into consecutive windows of a
// fixed duration, each window into steps of a fixed number of messages, and every
// window is padded to the same number of steps with all-zero messages (type 0:
// never processed), so that the windows form one fixed-shape array the step form
// replays with lob_step.
#include <cstring>
#include <vector>

#include "lob.h"

namespace {

constexpr int kFields = 8;

// window of a message time: -1 before the first window, n_windows past the last
int window_of(int32_t ts, int32_t start_s, int32_t window_s, int32_t n_windows) {
  if (ts < start_s) return -1;
  const long long k = ((long long)ts - start_s) / window_s;
  return k >= n_windows ? n_windows : (int)k;
}

}  // namespace

extern "C" {

lob_status lob_windows(const int32_t *msgs_host, int64_t n_msgs, int32_t start_s, int32_t window_s,
                       int32_t msgs_per_step, int32_t max_steps, int32_t n_windows, int32_t *out_host,
                       int32_t *steps_host, int64_t *first_host) {
  if (n_msgs < 0 || (n_msgs > 0 && !msgs_host) || window_s < 1 || msgs_per_step < 1 || max_steps < 0 ||
      n_windows < 1 || !steps_host || !first_host)
    return LOB_EINVAL;
  // first[k] = first message whose window is >= k; times must not decrease, so every
  // window is one contiguous run (messages before start_s belong to no window)
  std::vector<int64_t> first(n_windows + 1, n_msgs);
  int next = 0, last = -1;
  for (int64_t i = 0; i < n_msgs; ++i) {
    const int k = window_of(msgs_host[i * kFields + 6], start_s, window_s, n_windows);
    if (k < last) return LOB_EINVAL;  // a time went backwards across a window boundary
    last = k;
    while (next <= k && next <= n_windows) first[next++] = i;
  }
  lob_status st = LOB_OK;
  for (int k = 0; k < n_windows; ++k) {
    const int64_t cnt = first[k + 1] - first[k];
    const int64_t steps = (cnt + msgs_per_step - 1) / msgs_per_step;
    first_host[k] = first[k];
    steps_host[k] = (int32_t)(steps > max_steps ? max_steps : steps);
    if (steps > max_steps) st = LOB_ECAP;
    if (!out_host) continue;
    int32_t *w = out_host + (int64_t)k * max_steps * msgs_per_step * kFields;
    std::memset(w, 0, sizeof(int32_t) * (size_t)max_steps * msgs_per_step * kFields);
    const int64_t keep = cnt < (int64_t)max_steps * msgs_per_step ? cnt : (int64_t)max_steps * msgs_per_step;
    if (keep > 0) std::memcpy(w, msgs_host + first[k] * kFields, sizeof(int32_t) * (size_t)keep * kFields);
  }
  first_host[n_windows] = first[n_windows];
  return st;
}

}  // extern "C"
