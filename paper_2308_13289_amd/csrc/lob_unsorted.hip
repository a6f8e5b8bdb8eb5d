// lob_unsorted.hip -- the paper's book layout as a matching kernel (ablation).
//
// JAX-LOB keeps each side as a fixed-size array of orders in no particular order:
// an addition writes the first empty position, the best standing order is found
// by a search over the whole array for every trade, a cancel searches the array
// for its order id, and an order whose quantity reaches zero leaves an empty
// position behind (Section 4.1).  This kernel does the same on MI355X -- one
// wavefront per book, both sides in LDS as unsorted arrays, each search a
// wave-wide reduction -- so that the sorted layout of lob_kernels.hip and
// lob_small.hip can be measured against it on the same inputs.  Results are
// identical to theirs: priority among equal prices is the earlier (Ts, Tns), then
// arrival order, and the book goes back to HBM in priority order.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include "lob_device.h"
#include "lob_internal.h"

namespace lob {
namespace {

using namespace dev;

constexpr int kArrays = 7;  // P, Q, OID, TID, Ts, Tns, arrival rank

// One side in LDS: seven arrays of `cap` ints; a position with Q <= 0 is empty.
struct USide {
  int *P, *Q, *O, *T, *TS, *TNS, *AR;
};

__device__ __forceinline__ USide side_at(int *base, int cap, int sd) {
  int *b = base + (int64_t)sd * kArrays * cap;
  return {b, b + cap, b + 2 * cap, b + 3 * cap, b + 4 * cap, b + 5 * cap, b + 6 * cap};
}

// Priority key of an order: price, time and arrival rank.
struct Key {
  int p, ts, tns, a;
};

__device__ __forceinline__ Key key_at(const USide &S, int s) { return {S.P[s], S.TS[s], S.TNS[s], S.AR[s]}; }

// Is x ahead of y on side SD?  Better price, then earlier time, then earlier arrival.
template <int SD>
__device__ __forceinline__ bool ahead(const Key &x, const Key &y) {
  if (x.p != y.p) return SD == 1 ? x.p > y.p : x.p < y.p;
  if (x.ts != y.ts) return x.ts < y.ts;
  if (x.tns != y.tns) return x.tns < y.tns;
  return x.a < y.a;
}

__device__ __forceinline__ Key shfl_key(const Key &k, int o) {
  return {__shfl_xor(k.p, o, kWave), __shfl_xor(k.ts, o, kWave), __shfl_xor(k.tns, o, kWave),
          __shfl_xor(k.a, o, kWave)};
}

// The best live position of side SD among those with pred(s), -1 if none: a scan of
// the whole array (64 positions per step) and a butterfly over the wave.
template <int SD, typename Pred>
__device__ __forceinline__ int best_slot(const USide &S, int cap, Pred pred) {
  const int l = lane_id();
  Key bk = {0, 0, 0, INT_MAX};
  int bs = -1;
  for (int s = l; s < cap; s += kWave) {
    const int q = S.Q[s];
    if (q > 0 && pred(s)) {
      const Key k = key_at(S, s);
      if (bs < 0 || ahead<SD>(k, bk)) {
        bk = k;
        bs = s;
      }
    }
  }
  for (int o = 32; o >= 1; o >>= 1) {
    const Key ok = shfl_key(bk, o);
    const int os = __shfl_xor(bs, o, kWave);
    if (os >= 0 && (bs < 0 || ahead<SD>(ok, bk))) {
      bk = ok;
      bs = os;
    }
  }
  return uni(bs);
}

struct UBook {
  USide s[2];
  int cap;
  int arrival;  // rank of the next new order
};

// Matching loop of Section 4.1 against side OPP: one search for the best standing
// order per trade.
template <int OPP>
__device__ __forceinline__ int match(UBook &bk, State &st, int lim, int q, int a_oid, int a_tid, int ts, int tns) {
  const USide &S = bk.s[OPP];
  constexpr bool buyer = (OPP == 0);
  while (q > 0 && st.n[OPP] > 0) {
    const int b = best_slot<OPP>(S, bk.cap, [](int) { return true; });
    const int P = uni(S.P[b]), Q = uni(S.Q[b]);
    if (buyer ? P > lim : P < lim) break;
    const int f = min(q, Q);
    emit_one(st, P, f, uni(S.O[b]), a_oid, ts, tns, uni(S.T[b]), a_tid);
    st.traded_qty += f;
    st.n_trades++;
    if (lane_id() == 0) S.Q[b] = Q - f;
    if (Q == f) st.n[OPP]--;
    q -= f;
  }
  return q;
}

// Addition (Section 4.1, item 1): the first empty position.
template <int SD>
__device__ __forceinline__ void insert(UBook &bk, State &st, int P, int Q, int oid, int tid, int ts, int tns) {
  const USide &S = bk.s[SD];
  if (st.n[SD] >= st.cap) {
    st.rejected_qty += Q;
    st.flags |= kFlagSideFull;
    return;
  }
  const int l = lane_id();
  int e = -1;
  for (int base = 0; base < bk.cap; base += kWave) {
    const int s = base + l;
    const uint64_t m = ballot(s < bk.cap && S.Q[s] <= 0);
    if (m) {
      e = base + first_set(m);
      break;
    }
  }
  if (l == 0) {
    S.P[e] = P;
    S.Q[e] = Q;
    S.O[e] = oid;
    S.T[e] = tid;
    S.TS[e] = ts;
    S.TNS[e] = tns;
    S.AR[e] = bk.arrival;
  }
  bk.arrival++;
  st.n[SD]++;
}

// Cancel / delete (Section 4.1, item 2; Section 5.1.1 for initial orders).
template <int SD>
__device__ __forceinline__ void cancel(UBook &bk, State &st, int oid, int qty, int price) {
  if (qty <= 0) return;
  const USide &S = bk.s[SD];
  int b = best_slot<SD>(S, bk.cap, [&](int s) { return S.O[s] == oid; });
  if (b < 0) b = best_slot<SD>(S, bk.cap, [&](int s) { return S.O[s] <= -9000 && S.P[s] == price; });
  if (b < 0) {
    st.cancel_miss++;
    return;
  }
  const int Q = uni(S.Q[b]);
  st.cancelled_qty += min(qty, Q);
  const int left = Q - qty;
  if (lane_id() == 0) S.Q[b] = left > 0 ? left : 0;
  if (left <= 0) st.n[SD]--;
}

// L2 of side SD: level k is the best price strictly behind level k-1, with the sum
// of its orders' quantities.
template <int SD>
__device__ __forceinline__ void l2_side(const UBook &bk, int L, int2 *out) {
  const USide &S = bk.s[SD];
  const int l = lane_id();
  bool have_prev = false;
  int prev = 0;
  for (int lev = 0; lev < L; ++lev) {
    int px = 0;
    bool found = false;
    for (int s = l; s < bk.cap; s += kWave) {
      const int p = S.P[s];
      if (S.Q[s] > 0 && (!have_prev || (SD == 1 ? p < prev : p > prev)) &&
          (!found || (SD == 1 ? p > px : p < px))) {
        px = p;
        found = true;
      }
    }
    for (int o = 32; o >= 1; o >>= 1) {
      const int op = __shfl_xor(px, o, kWave);
      const int of = __shfl_xor(found ? 1 : 0, o, kWave);
      if (of && (!found || (SD == 1 ? op > px : op < px))) {
        px = op;
        found = true;
      }
    }
    if (!uni(found ? 1 : 0)) {
      if (l == 0) out[lev] = make_int2(-1, 0);
      continue;
    }
    px = uni(px);
    // the level's exact sum (64-bit), reported capped at INT_MAX
    long long qs = 0;
    for (int s = l; s < bk.cap; s += kWave)
      if (S.Q[s] > 0 && S.P[s] == px) qs += S.Q[s];
    for (int o = 32; o >= 1; o >>= 1)
      qs += ((long long)__shfl_xor((int)(qs >> 32), o, kWave) << 32) | (unsigned)__shfl_xor((int)(unsigned)qs, o, kWave);
    if (l == 0) out[lev] = make_int2(px, qs > INT_MAX ? INT_MAX : (int)qs);
    prev = px;
    have_prev = true;
  }
}

__device__ __forceinline__ void write_l2(const UBook &bk, int L, int32_t *row) {
  int2 *o = reinterpret_cast<int2 *>(row);
  l2_side<0>(bk, L, o);
  l2_side<1>(bk, L, o + L);
}

__device__ __forceinline__ void process_msg(UBook &bk, State &st, int code, int P, int Q, int oid, int tid, int ts,
                                            int tns) {
  if (code == 0) return;
  const bool buys = (code & 1) == 0;
  if (code <= 4) {
    const bool limit = code <= 2;
    if (Q > 0) {
      if (limit)
        st.limit_qty += Q;
      else
        st.market_qty += Q;
    }
    const int lim = limit ? P : (buys ? INT_MAX : 0);
    const int rem = buys ? match<0>(bk, st, lim, Q, oid, tid, ts, tns) : match<1>(bk, st, lim, Q, oid, tid, ts, tns);
    if (rem > 0) {
      if (!limit)
        st.market_discarded += rem;
      else if (buys)
        insert<1>(bk, st, P, rem, oid, tid, ts, tns);
      else
        insert<0>(bk, st, P, rem, oid, tid, ts, tns);
    }
  } else if (buys) {
    cancel<1>(bk, st, oid, Q, P);
  } else {
    cancel<0>(bk, st, oid, Q, P);
  }
}

__device__ void run_book(const ProcArgs &a, int i, int *lds) {
  const int l = lane_id();
  const int book = a.book_ids ? uni(a.book_ids[i]) : i;
  if (book < 0 || book >= a.n_total) return;
  BookHdr *h = a.hdr + book;
  State st;
  st.n[0] = uni(h->n[0]);
  st.n[1] = uni(h->n[1]);
  st.cap = uni(h->cap);
  if (2 * kArrays * st.cap > 2 * a.lds_int2_per_wave) {  // above the launch's capacity bound: left untouched
    if (l == 0) h->flags |= kFlagBadLoad;
    return;
  }
  st.flags = uni(h->flags);
  st.n_msgs = uni64(h->n_msgs);
  st.n_trades = uni64(h->n_trades);
  st.limit_qty = uni64(h->limit_qty);
  st.market_qty = uni64(h->market_qty);
  st.traded_qty = uni64(h->traded_qty);
  st.cancelled_qty = uni64(h->cancelled_qty);
  st.market_discarded = uni64(h->market_discarded);
  st.rejected_qty = uni64(h->rejected_qty);
  st.cancel_miss = uni64(h->cancel_miss);
  st.last_ts = uni(h->last_ts);
  st.last_tns = uni(h->last_tns);
  st.seen = uni(h->seen_time);
  st.log_cap = uni64(h->log_cap);
  st.log_count = uni64(h->log_count);
  st.log = a.log ? a.log + uni64(h->log_off) * kTradeFields : nullptr;
  const int row = a.out_rows ? uni(a.out_rows[i]) : i;
  st.fills = a.fills ? a.fills + (int64_t)row * a.fill_cap * kTradeFields : nullptr;
  st.fill_cap = a.fill_cap;
  st.fill_count = 0;
  st.agent_tid = a.agent_tid;

  UBook bk;
  bk.cap = st.cap;
  bk.s[0] = side_at(lds, st.cap, 0);
  bk.s[1] = side_at(lds, st.cap, 1);
  bk.arrival = st.cap;  // above every loaded order's rank
  int2 *hb = a.books + uni64(h->book_off);
  // the book arrives in priority order: position = rank
  for (int sd = 0; sd < 2; ++sd) {
    const USide &S = bk.s[sd];
    for (int s = l; s < st.cap; s += kWave) {
      if (s < st.n[sd]) {
        const int2 pq = hb[(int64_t)(sd * 3 + 0) * st.cap + s];
        const int2 ot = hb[(int64_t)(sd * 3 + 1) * st.cap + s];
        const int2 tt = hb[(int64_t)(sd * 3 + 2) * st.cap + s];
        S.P[s] = pq.x;
        S.Q[s] = pq.y;
        S.O[s] = ot.x;
        S.T[s] = ot.y;
        S.TS[s] = tt.x;
        S.TNS[s] = tt.y;
        S.AR[s] = s;
      } else {
        S.Q[s] = 0;
      }
    }
  }

  long long beg1 = 0, n1 = 0;
  if (a.msgs) {
    if (a.ranges) {
      beg1 = a.ranges[2 * i];
      n1 = a.ranges[2 * i + 1] - beg1;
    } else if (a.offs) {
      beg1 = a.offs[i];
      n1 = a.offs[i + 1] - beg1;
    } else {
      beg1 = (long long)i * a.w1;
      n1 = a.w1;
    }
  }
  const long long n2 = (a.msgs2 && a.w2 > 0) ? a.w2 : 0;
  const long long beg2 = (long long)i * a.w2;
  int32_t *l2_rows = a.l2_mode != 1 ? nullptr
                     : a.l2_stride ? a.l2_out + (int64_t)i * a.l2_stride : a.l2_out + beg1 * 4 * a.levels;
  const long long total = n1 + n2;
  for (long long k0 = 0; k0 < total; k0 += kWave) {
    const int cnt = (int)((total - k0) < kWave ? (total - k0) : kWave);
    int4 u = make_int4(0, 0, 0, 0), v = make_int4(0, 0, 0, 0);
    if (l < cnt) {
      const long long k = k0 + l;
      const int32_t *rec = k < n1 ? a.msgs + (beg1 + k) * kMsgFields : a.msgs2 + (beg2 + k - n1) * kMsgFields;
      u = reinterpret_cast<const int4 *>(rec)[0];
      v = reinterpret_cast<const int4 *>(rec)[1];
    }
    const bool ok = (l < cnt) & (u.x >= 1) & (u.x <= 4) & ((u.y == 1) | (u.y == -1));
    const int code = !ok ? 0 : (u.x == 1 ? 1 : u.x == 4 ? 3 : 5) + (u.y == 1 ? 1 : 0);
    const uint64_t vmask = ballot(ok);
    if (vmask) {
      const uint64_t below = vmask & mask_lt();
      const int src = below ? 63 - __builtin_clzll(below) : 0;
      const int pts = from_lane(v.z, src), ptns = from_lane(v.w, src);
      const bool has_prev = below != 0 || st.seen;
      const int cts = below ? pts : st.last_ts, ctns = below ? ptns : st.last_tns;
      const bool dec = ok & has_prev & ((v.z < cts) | ((v.z == cts) & (v.w < ctns)));
      if (ballot(dec)) st.flags |= kFlagTimeOrder;
      const int top = 63 - __builtin_clzll(vmask);
      st.last_ts = rdlane(v.z, top);
      st.last_tns = rdlane(v.w, top);
      st.seen = 1;
    }
    st.n_msgs += cnt;
    for (int j = 0; j < cnt; ++j) {
      process_msg(bk, st, rdlane(code, j), rdlane(u.z, j), rdlane(u.w, j), rdlane(v.x, j), rdlane(v.y, j),
                  rdlane(v.z, j), rdlane(v.w, j));
      if (l2_rows && k0 + j < n1) write_l2(bk, a.levels, l2_rows + (k0 + j) * 4 * a.levels);
    }
  }
  if (a.l2_mode == 2) write_l2(bk, a.levels, a.l2_out + (int64_t)row * 4 * a.levels);

  // back to HBM in priority order: a live position's rank is the number of live
  // positions ahead of it
  for (int sd = 0; sd < 2; ++sd) {
    const USide &S = bk.s[sd];
    for (int s = l; s < st.cap; s += kWave) {
      const int q = S.Q[s];
      if (q <= 0) continue;
      const Key me = key_at(S, s);
      int r = 0;
      for (int t = 0; t < st.cap; ++t) {
        if (S.Q[t] <= 0) continue;
        r += sd == 1 ? ahead<1>(key_at(S, t), me) : ahead<0>(key_at(S, t), me);
      }
      const int p = me.p;
      hb[(int64_t)(sd * 3 + 0) * st.cap + r] = make_int2(p, q);
      hb[(int64_t)(sd * 3 + 1) * st.cap + r] = make_int2(S.O[s], S.T[s]);
      hb[(int64_t)(sd * 3 + 2) * st.cap + r] = make_int2(S.TS[s], S.TNS[s]);
    }
  }
  if (st.fills) {
    if (st.fill_count > st.fill_cap) st.flags |= kFlagFillsFull;
    if (l == 0 && a.fill_counts) a.fill_counts[row] = st.fill_count;
  }
  if (l == 0) {
    h->n[0] = st.n[0];
    h->n[1] = st.n[1];
    h->flags = st.flags;
    h->n_msgs = st.n_msgs;
    h->n_trades = st.n_trades;
    h->limit_qty = st.limit_qty;
    h->market_qty = st.market_qty;
    h->traded_qty = st.traded_qty;
    h->cancelled_qty = st.cancelled_qty;
    h->market_discarded = st.market_discarded;
    h->rejected_qty = st.rejected_qty;
    h->cancel_miss = st.cancel_miss;
    h->last_ts = st.last_ts;
    h->last_tns = st.last_tns;
    h->seen_time = st.seen;
    h->log_count = st.log_count;
  }
}

__global__ void __launch_bounds__(1024) k_process_unsorted(ProcArgs a) {
  extern __shared__ int usmem[];
  const int w = uni(threadIdx.x / kWave);  // uniform: one wave = one book
  const int i = blockIdx.x * a.bpb + w;
  if (i >= a.n) return;
  run_book(a, i, usmem + (int64_t)w * a.lds_int2_per_wave * 2);
}

}  // namespace

// ints of LDS one wave needs for books of capacity <= cap
int unsorted_lds_ints(int cap) { return 2 * kArrays * cap; }

hipError_t launch_process_unsorted(const ProcArgs &a, hipStream_t s) {
  const int threads = a.bpb * kWave;
  const size_t lds = (size_t)a.bpb * a.lds_int2_per_wave * sizeof(int2);
  const int grid = (a.n + a.bpb - 1) / a.bpb;
  hipLaunchKernelGGL(k_process_unsorted, dim3(grid), dim3(threads), lds, s, a);
  return hipGetLastError();
}

hipError_t set_process_unsorted_lds_limit(size_t bytes) {
  return hipFuncSetAttribute((const void *)k_process_unsorted, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

}  // namespace lob
