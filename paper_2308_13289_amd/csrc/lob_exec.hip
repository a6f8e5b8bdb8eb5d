// lob_exec.hip -- the execution environment around the matcher (JAX-LOB Section 5.2).
//
// k_exec_prepare runs before the matching launch: it turns each book's action
// (order sizes at four reference prices, Section 5.2.3) into agent orders, or
// into the forced market order of Section 5.2.5, and notes where the step's trades
// will start in the book's trade log.  k_exec_finish runs after it: the
// observation vector of Section 5.2.2 from the level-1 rows the matcher left in
// the observation buffer, the reward of eqs. (rewardfunc) and (vwap) from the
// step's logged trades and agent fills, and the task state.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lob.h"
#include "lob_device.h"
#include "lob_internal.h"

static_assert(sizeof(lob_exec_state) == 48, "lob_exec_state layout");

namespace lob {
namespace {

using namespace dev;

constexpr int kActs = 4;  // orders an action can make

// time of the step's last data message (types 1..4), else the book's last time
__device__ __forceinline__ int2 step_time(const int32_t *win, int W, const BookHdr *h) {
  for (int k = W - 1; k >= 0; --k) {
    const int32_t *m = win + (int64_t)k * kMsgFields;
    if (m[0] >= 1 && m[0] <= 4) return make_int2(m[6], m[7]);
  }
  return make_int2(h->last_ts, h->last_tns);
}

// One thread per listed book.
__global__ void __launch_bounds__(256) k_exec_prepare(const BookHdr *hdr, const int2 *books, const int32_t *ids,
                                                      int n, int n_total, const int32_t *window, int W,
                                                      const int32_t *action_qty, lob_exec_params p,
                                                      lob_exec_state *state, int32_t *acts, int64_t *aux) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t *out = acts + (int64_t)i * kActs * kMsgFields;
  for (int k = 0; k < kActs * kMsgFields; ++k) out[k] = 0;  // type 0: no order
  const int b = ids ? ids[i] : i;
  if (b < 0 || b >= n_total) {
    aux[2 * i] = aux[2 * i + 1] = 0;
    return;
  }
  const BookHdr *h = hdr + b;
  aux[2 * i] = h->log_count;  // the step's trades start here in the log
  aux[2 * i + 1] = h->n_trades;
  lob_exec_state s = state[i];
  const int rem = s.task_qty - s.exec_qty;
  if (s.done || rem <= 0) return;
  const int2 t = step_time(window + (int64_t)i * W * kMsgFields, W, h);
  const int side = s.task_side == 1 ? 1 : -1;
  int oid = s.next_oid;
  if (t.x >= s.end_s - 60) {
    // one minute before the end: the remaining quantity as a market order
    const int32_t m[kMsgFields] = {4, side, 0, rem, oid++, p.agent_tid, t.x, t.y};
    for (int f = 0; f < kMsgFields; ++f) out[f] = m[f];
  } else {
    const int cap = h->cap;
    const int2 *bk = books + h->book_off;
    const int ask = h->n[0] > 0 ? bk[0].x : -1;                // best ask: slot 0 of side 0
    const int bid = h->n[1] > 0 ? bk[3 * (int64_t)cap].x : -1;  // best bid: slot 0 of side 1
    const int far = side == 1 ? ask : bid;
    const int near = side == 1 ? bid : ask;
    const int mid = (ask >= 0 && bid >= 0) ? (int)(((long long)ask + bid) >> 1) : -1;
    const long long pas = (long long)near + (long long)(side == 1 ? -1 : 1) * p.passive_ticks * p.tick;
    const int passive = (near >= 0 && pas > 0 && pas <= INT32_MAX) ? (int)pas : -1;
    const int px[kActs] = {far, mid, near, passive};
    int r = 0;
    for (int k = 0; k < kActs; ++k) {
      const int q = action_qty[(int64_t)i * kActs + k];
      if (q <= 0 || px[k] <= 0) continue;
      const int32_t m[kMsgFields] = {1, side, px[k], q, oid++, p.agent_tid, t.x, t.y};
      for (int f = 0; f < kMsgFields; ++f) out[r * kMsgFields + f] = m[f];
      ++r;
    }
  }
  state[i].next_oid = oid;
}

// int64 sum over the wave
__device__ __forceinline__ long long wave_sum64(long long v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// One wave per listed book.
__global__ void __launch_bounds__(256) k_exec_finish(BookHdr *hdr, const int32_t *ids, int n, int n_total,
                                                     const int32_t *log, const int32_t *window, int W,
                                                     lob_exec_params p, lob_exec_state *state, int32_t *obs,
                                                     double *reward, const int32_t *fills, int F,
                                                     const int32_t *fill_counts, const int64_t *aux) {
  const int w = uni(threadIdx.x / kWave);  // uniform: one wave = one book
  const int i = blockIdx.x * 4 + w;
  if (i >= n) return;
  const int l = lane_id();
  const int b = ids ? uni(ids[i]) : i;
  if (b < 0 || b >= n_total) return;
  BookHdr *h = hdr + b;
  lob_exec_state s = state[i];
  const int sell = s.task_side == 1 ? 0 : 1;
  int32_t *o = obs + (int64_t)i * (6 * W + 8);
  // the matcher left the level-1 row (ask P, ask Q, bid P, bid Q) of data message k
  // at o[4k .. 4k+4); read them all before the observation overwrites them
  constexpr int kMaxChunks = 4;  // W <= 256
  int ap[kMaxChunks], aq[kMaxChunks], bp[kMaxChunks], bq[kMaxChunks];
#pragma unroll
  for (int c = 0; c < kMaxChunks; ++c) {
    const int k = c * kWave + l;
    ap[c] = aq[c] = bp[c] = bq[c] = 0;
    if (k < W) {
      ap[c] = o[4 * k];
      aq[c] = o[4 * k + 1];
      bp[c] = o[4 * k + 2];
      bq[c] = o[4 * k + 3];
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  int last_mid = -1;
#pragma unroll
  for (int c = 0; c < kMaxChunks; ++c) {
    const int k = c * kWave + l;
    const bool has_a = aq[c] > 0, has_b = bq[c] > 0;
    const int askp = has_a ? ap[c] : -1, bidp = has_b ? bp[c] : -1;
    const int mid = (has_a && has_b) ? (int)(((long long)askp + bidp) >> 1) : -1;
    const int near = sell ? askp : bidp;
    const long long pas = (long long)near + (long long)(sell ? 1 : -1) * p.passive_ticks * p.tick;
    const int passive = (near >= 0 && pas > 0 && pas <= INT32_MAX) ? (int)pas : -1;
    const int spread = (has_a && has_b) ? askp - bidp : -1;
    const int imb = (has_a ? aq[c] : 0) - (has_b ? bq[c] : 0);
    if (k < W) {
      o[k] = bidp;
      o[W + k] = askp;
      o[2 * W + k] = mid;
      o[3 * W + k] = passive;
      o[4 * W + k] = spread;
      o[5 * W + k] = imb;
    }
    if (c * kWave <= W - 1 && W - 1 < (c + 1) * kWave) last_mid = rdlane(mid, (W - 1) - c * kWave);
  }
  // all trades of the step: the log records appended since k_exec_prepare
  const long long before = aux[2 * i], after = h->log_count;
  long long sqp = 0, sq = 0;
  if (log) {
    const int32_t *rec = log + h->log_off * kTradeFields;
    for (long long r = before + l; r < after; r += kWave) {
      const int32_t *t = rec + r * kTradeFields;
      sqp += (long long)t[0] * t[1];
      sq += t[1];
    }
  }
  sqp = wave_sum64(sqp);
  sq = wave_sum64(sq);
  if (l != 0) return;
  // the agent's fills of the step, in order, counted up to the task size
  const int nf = min(fill_counts[i], F);
  long long A = 0, B = 0;
  int exec = s.exec_qty;
  for (int j = 0; j < nf; ++j) {
    const int32_t *f = fills + ((int64_t)i * F + j) * kTradeFields;
    const int take = min(f[1], s.task_qty - exec);
    if (take <= 0) continue;
    A += (long long)take * f[0];
    B += take;
    exec += take;
  }
  // fills past the buffer count only if the stored ones left the task unfinished
  int flags = s.flags;
  if (fill_counts[i] > F && exec < s.task_qty) flags |= LOB_EXEC_FILLS_MISSING;
  double R = 0.0;
  if (sq > 0) {
    const double vwap = (double)sqp / (double)sq;
    const double bv = (double)B * vwap;
    R = ((double)A - bv) + p.lambda * (bv - (double)B * (double)s.p_init);
  }
  reward[i] = R;
  const int2 t = step_time(window + (int64_t)i * W * kMsgFields, W, h);
  int es = t.x - s.start_s, ens = t.y - s.start_ns;
  if (ens < 0) {
    ens += 1000000000;
    es -= 1;
  }
  int32_t *tail = o + 6 * W;
  tail[0] = t.x;
  tail[1] = t.y;
  tail[2] = es;
  tail[3] = ens;
  tail[4] = s.p_init;
  tail[5] = last_mid >= 0 ? last_mid - s.p_init : 0;
  tail[6] = s.task_qty;
  tail[7] = exec;
  state[i].exec_qty = exec;
  state[i].revenue = s.revenue + A;
  state[i].done = (exec >= s.task_qty || t.x >= s.end_s) ? 1 : 0;
  // trades of the step that found no room in the log
  if (h->n_trades - aux[2 * i + 1] > after - before) flags |= LOB_EXEC_TRADES_MISSING;
  state[i].flags = flags;
  if (!p.keep_trades && log) h->log_count = before;
}

}  // namespace

hipError_t launch_exec_prepare(const BookHdr *hdr, const int2 *books, const int32_t *ids, int n, int n_total,
                               const int32_t *window, int W, const int32_t *action_qty, const lob_exec_params &p,
                               lob_exec_state *state, int32_t *acts, int64_t *aux, hipStream_t s) {
  hipLaunchKernelGGL(k_exec_prepare, dim3((n + 255) / 256), dim3(256), 0, s, hdr, books, ids, n, n_total, window, W,
                     action_qty, p, state, acts, aux);
  return hipGetLastError();
}

hipError_t launch_exec_finish(BookHdr *hdr, const int32_t *ids, int n, int n_total, const int32_t *log,
                              const int32_t *window, int W, const lob_exec_params &p, lob_exec_state *state,
                              int32_t *obs, double *reward, const int32_t *fills, int F, const int32_t *fill_counts,
                              const int64_t *aux, hipStream_t s) {
  hipLaunchKernelGGL(k_exec_finish, dim3((n + 3) / 4), dim3(256), 0, s, hdr, ids, n, n_total, log, window, W, p,
                     state, obs, reward, fills, F, fill_counts, aux);
  return hipGetLastError();
}

}  // namespace lob
