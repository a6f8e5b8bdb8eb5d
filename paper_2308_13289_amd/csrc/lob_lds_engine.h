// lob_lds_engine.h -- the matching engine of lob_kernels.hip: one wavefront per book,
// each side kept SORTED in price-time priority (slot 0 = best) as three arrays of
// int2 pairs -- (P, Q), (OID, TID), (Ts, Tns) -- in LDS, with the slots past the LDS
// window W in the book's HBM arrays (SPILL).  Included by lob_kernels.hip (the LDS
// kernel) and by lob_small.hip, whose register kernel hands a book whose times went
// backwards to it with W = 0 (every slot in HBM): this engine keeps each order's
// time beside it and places a new order by price and time.
#pragma once
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include "lob_device.h"
#include "lob_internal.h"

namespace lob {
namespace lds {

using namespace dev;

// ---------------------------------------------------------------- book storage

template <bool SPILL>
struct View {
  int2 *lds;   // [2][3][W]
  int2 *hbm;   // [2][3][cap]
  int W, cap;
  __device__ __forceinline__ int2 *at(int sd, int p, int s) const {
    if constexpr (!SPILL) {
      return lds + (sd * 3 + p) * W + s;
    } else {
      return s < W ? lds + (sd * 3 + p) * W + s : hbm + (int64_t)(sd * 3 + p) * cap + s;
    }
  }
};

// Make the vector-memory stores of this wave visible to its later loads before
// moving on (only needed when book slots live in HBM).
template <bool SPILL>
__device__ __forceinline__ void spill_fence() {
  if constexpr (SPILL) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// Slots [from+m, n) move to [from, n-m).
template <bool SPILL>
__device__ void shift_down(const View<SPILL> &B, int sd, int from, int m, int n) {
  const int l = lane_id();
  for (int base = from & ~63; base < n - m; base += kWave) {
    const int s = base + l;
    const bool act = s >= from && s < n - m;
    int2 a, b, c;
    if (act) {
      a = *B.at(sd, 0, s + m);
      b = *B.at(sd, 1, s + m);
      c = *B.at(sd, 2, s + m);
    }
    if (act) {
      *B.at(sd, 0, s) = a;
      *B.at(sd, 1, s) = b;
      *B.at(sd, 2, s) = c;
    }
    spill_fence<SPILL>();
  }
}

// Slots [pos, n) move to [pos+1, n+1); chunks are taken from the top down.
template <bool SPILL>
__device__ void shift_up(const View<SPILL> &B, int sd, int pos, int n) {
  const int l = lane_id();
  for (int base = (n - 1) & ~63; base >= (pos & ~63); base -= kWave) {
    const int s = base + l;
    const bool act = s >= pos && s < n;
    int2 a, b, c;
    if (act) {
      a = *B.at(sd, 0, s);
      b = *B.at(sd, 1, s);
      c = *B.at(sd, 2, s);
    }
    if (act) {
      *B.at(sd, 0, s + 1) = a;
      *B.at(sd, 1, s + 1) = b;
      *B.at(sd, 2, s + 1) = c;
    }
    spill_fence<SPILL>();
  }
}

// Slot 0 (the best order) of a side, kept in scalar registers so that the common
// cases -- a limit that does not cross, an aggressor filled by the best order
// alone, a cancel of the best order -- need no pass over the side.
template <bool SPILL>
__device__ __forceinline__ void load_best(const View<SPILL> &B, State &st, int sd) {
  if (st.n[sd] > 0) {
    const int2 pq = *B.at(sd, 0, 0);
    const int2 ot = *B.at(sd, 1, 0);
    st.bP[sd] = uni(pq.x);
    st.bQ[sd] = uni(pq.y);
    st.bO[sd] = uni(ot.x);
    st.bT[sd] = uni(ot.y);
  }
}

// Matching loop of Section 4.1 against side OPP (0 asks, 1 bids) for an aggressor
// with limit price lim and quantity q.  Returns the unfilled quantity.
template <int OPP, bool SPILL>
__device__ __forceinline__ int match(const View<SPILL> &B, State &st, int lim, int q, int a_oid, int a_tid,
                                     int ts, int tns) {
  const int n = st.n[OPP];
  constexpr bool buyer = (OPP == 0);
  if (q <= 0 || n == 0) return q;
  if (buyer ? st.bP[OPP] > lim : st.bP[OPP] < lim) return q;  // the best standing price does not overlap
  if (q <= st.bQ[OPP]) {
    // Q_s' = Q_s - Q_a >= 0: one trade with the best order, the aggressor is done
    emit_one(st, st.bP[OPP], q, st.bO[OPP], a_oid, ts, tns, st.bT[OPP], a_tid);
    st.traded_qty += q;
    st.n_trades++;
    if (q < st.bQ[OPP]) {
      st.bQ[OPP] -= q;
      if (lane_id() == 0) *B.at(OPP, 0, 0) = make_int2(st.bP[OPP], st.bQ[OPP]);
      spill_fence<SPILL>();
    } else {
      shift_down(B, OPP, 0, 1, n);
      st.n[OPP] = n - 1;
      load_best(B, st, OPP);
    }
    return 0;
  }
  // the aggressor outlasts the best order: one prefix scan per 64 crossing orders
  const int l = lane_id();
  int removed = 0;
  for (int base = 0; base < n && q > 0; base += kWave) {
    const int s = base + l;
    const bool valid = s < n;
    int2 pq = make_int2(0, 0);
    if (valid) pq = *B.at(OPP, 0, s);
    const bool cross = valid && (buyer ? pq.x <= lim : pq.x >= lim);
    const int qv = cross ? pq.y : 0;
    // running sums of the crossing quantities; excl is exact wherever it is below q
    int incl, excl;
    if (q < kScanExactQ) {
      const int qc = min(qv, q + 1);
      incl = scan_incl(qc);
      excl = incl - qc;
    } else {
      incl = scan_incl_sat(qv);
      excl = shr1(incl, 0);
    }
    const bool takes = cross && excl < q;
    const uint64_t mt = ballot(takes);
    if (mt == 0) break;
    const int ntr = popc(mt);
    const int room = q - excl;
    const bool full = takes && qv <= room;
    const int nfull = popc(ballot(full));
    int fill = 0;
    int2 ot = make_int2(0, 0);
    if (takes) {
      fill = min(qv, room);
      ot = *B.at(OPP, 1, s);
      if (!full) *B.at(OPP, 0, s) = make_int2(pq.x, pq.y - fill);
    }
    emit(st, takes, ntr, pq.x, fill, ot.x, a_oid, ts, tns, ot.y, a_tid);
    const int consumed = (nfull == ntr) ? rdlane(incl, ntr - 1) : q;
    st.traded_qty += consumed;
    st.n_trades += ntr;
    q -= consumed;
    removed += nfull;
    if (nfull < kWave) break;
  }
  spill_fence<SPILL>();
  if (removed > 0) {
    shift_down(B, OPP, 0, removed, n);
    st.n[OPP] = n - removed;
  }
  load_best(B, st, OPP);
  return q;
}

// Add (Section 4.1, item 1) on side SD: the new order goes to its price-time
// position.  While a book's times have never gone backwards every standing order is
// at most as old as the new one, so that position is behind every order with an
// equal or better price; in a book flagged for times going backwards the times of
// the orders at the new order's price are compared too (equal times: the standing
// order arrived first).
template <int SD, bool SPILL>
__device__ __forceinline__ void insert(const View<SPILL> &B, State &st, int P, int Q, int oid, int tid, int ts,
                                       int tns) {
  const int l = lane_id();
  const int n = st.n[SD];
  if (n >= st.cap) {
    st.rejected_qty += Q;
    st.flags |= kFlagSideFull;
    return;
  }
  const bool timed = (st.flags & kFlagTimeOrder) != 0;
  int pos = 0;
  // strictly better than the best order: it becomes slot 0, no search needed
  if (n > 0 && !(SD == 1 ? P > st.bP[SD] : P < st.bP[SD])) {
    for (int base = 0; base < n; base += kWave) {
      const int s = base + l;
      bool ahead = false;
      if (s < n) {
        const int p = B.at(SD, 0, s)->x;
        ahead = (SD == 1) ? p >= P : p <= P;
        if (timed && p == P) {
          const int2 t = *B.at(SD, 2, s);
          ahead = t.x < ts || (t.x == ts && t.y <= tns);
        }
      }
      const int k = popc(ballot(ahead));
      pos += k;
      if (k < kWave) break;
    }
  }
  if (pos < n) shift_up(B, SD, pos, n);
  if (l == 0) {
    *B.at(SD, 0, pos) = make_int2(P, Q);
    *B.at(SD, 1, pos) = make_int2(oid, tid);
    *B.at(SD, 2, pos) = make_int2(ts, tns);
  }
  spill_fence<SPILL>();
  st.n[SD] = n + 1;
  if (pos == 0) {
    st.bP[SD] = P;
    st.bQ[SD] = Q;
    st.bO[SD] = oid;
    st.bT[SD] = tid;
  }
}

// Cancel / delete (Section 4.1, item 2; Section 5.1.1 for initial orders) on side SD.
template <int SD, bool SPILL>
__device__ __forceinline__ void cancel(const View<SPILL> &B, State &st, int oid, int qty, int price) {
  if (qty <= 0) return;
  const int l = lane_id();
  const int n = st.n[SD];
  if (n == 0) {
    st.cancel_miss++;
    return;
  }
  int k = -1;
  if (st.bO[SD] == oid) {
    k = 0;  // the best order: the first order with this id in priority order
  } else {
    for (int base = 0; base < n; base += kWave) {
      const int s = base + l;
      bool hit = false;
      if (s < n) hit = B.at(SD, 1, s)->x == oid;
      const uint64_t m = ballot(hit);
      if (m) {
        k = base + first_set(m);
        break;
      }
    }
    if (k < 0) {
      for (int base = 0; base < n; base += kWave) {
        const int s = base + l;
        bool hit = false;
        if (s < n) hit = B.at(SD, 1, s)->x <= -9000 && B.at(SD, 0, s)->x == price;
        const uint64_t m = ballot(hit);
        if (m) {
          k = base + first_set(m);
          break;
        }
      }
    }
  }
  if (k < 0) {
    st.cancel_miss++;
    return;
  }
  const int2 pq = *B.at(SD, 0, k);
  const int P = uni(pq.x), Q = uni(pq.y);
  st.cancelled_qty += min(qty, Q);
  const int left = Q - qty;
  if (left > 0) {
    if (l == 0) *B.at(SD, 0, k) = make_int2(P, left);
    spill_fence<SPILL>();
    if (k == 0) st.bQ[SD] = left;
  } else {
    shift_down(B, SD, k, 1, n);
    st.n[SD] = n - 1;
    if (k == 0) load_best(B, st, SD);
  }
}

// L2 of one side: the first L distinct prices with their summed quantities into
// out[0..L) as (price, qty); missing levels (-1, 0).  A level is a run of equal
// prices in priority order; its quantity is the exact sum of the run, capped at
// INT_MAX (level_qty).
template <bool SPILL>
__device__ void l2_side(const View<SPILL> &B, const State &st, int sd, int L, int2 *out) {
  const int l = lane_id();
  const int n = st.n[sd];
  int levels = 0;
  long long carry = 0;
  for (int base = 0; base < n && levels < L; base += kWave) {
    const int s = base + l;
    const bool valid = s < n;
    int2 pq = make_int2(0, 0);
    int next = 0;
    if (valid) {
      pq = *B.at(sd, 0, s);
      if (s + 1 < n) next = B.at(sd, 0, s + 1)->x;
    }
    const bool is_last = valid && (s + 1 == n || next != pq.x);
    const uint64_t ml = ballot(is_last);
    const int lq = level_qty(valid ? pq.y : 0, ml, carry);
    const int lev = levels + popc(ml & mask_lt());
    if (is_last && lev < L) out[lev] = make_int2(pq.x, lq);
    levels += popc(ml);
  }
  const int have = levels < L ? levels : L;
  if (l >= have && l < L) out[l] = make_int2(-1, 0);
}

template <bool SPILL>
__device__ __forceinline__ void write_l2(const View<SPILL> &B, const State &st, int L, int32_t *row) {
  int2 *o = reinterpret_cast<int2 *>(row);
  l2_side(B, st, 0, L, o);
  l2_side(B, st, 1, L, o + L);
}

// One message (Section 4.2) given its case code (see process_all).
template <bool SPILL>
__device__ __forceinline__ void process_msg(const View<SPILL> &B, State &st, int code, int P, int Q, int oid,
                                            int tid, int ts, int tns) {
  if (code == 0) return;  // padding / unknown type or side: never processed
  const bool buys = (code & 1) == 0;  // even codes are buy-side messages
  if (code <= 4) {
    // limit (1, 2): match, then rest the remainder as one new order (item 1);
    // market (3, 4): match at price 0 (sell) / max_int (buy), drop the rest (item 3)
    const bool limit = code <= 2;
    if (Q > 0) {
      if (limit)
        st.limit_qty += Q;
      else
        st.market_qty += Q;
    }
    const int lim = limit ? P : (buys ? INT_MAX : 0);
    const int rem = buys ? match<0>(B, st, lim, Q, oid, tid, ts, tns) : match<1>(B, st, lim, Q, oid, tid, ts, tns);
    if (rem > 0) {
      if (!limit)
        st.market_discarded += rem;
      else if (buys)
        insert<1>(B, st, P, rem, oid, tid, ts, tns);
      else
        insert<0>(B, st, P, rem, oid, tid, ts, tns);
    }
  } else {
    // cancel and delete (5, 6) are the same operation (item 2)
    if (buys)
      cancel<1>(B, st, oid, Q, P);
    else
      cancel<0>(B, st, oid, Q, P);
  }
}

// The book's messages: source 1 msgs[beg1, beg1 + n1), then source 2 (the step
// form's agent orders) msgs2[beg2, beg2 + n2).  They are read in 64-message chunks,
// one record per lane; per chunk the lanes work out each message's case code
// (1/2 limit sell/buy, 3/4 market sell/buy, 5/6 cancel-or-delete on the ask/bid
// side, 0 skipped), the message count and the check that valid messages' times do
// not decrease, so the scalar path per message only dispatches.
template <bool SPILL>
__device__ __forceinline__ void process_all(const View<SPILL> &B, State &st, const ProcArgs &a, long long beg1,
                                            long long n1, long long beg2, long long n2, int32_t *l2_rows) {
  const int l = lane_id();
  const long long total = n1 + n2;
  for (long long k0 = 0; k0 < total; k0 += kWave) {
    const int cnt = (int)((total - k0) < kWave ? (total - k0) : kWave);
    int4 u = make_int4(0, 0, 0, 0), v = make_int4(0, 0, 0, 0);
    if (l < cnt) {
      const long long k = k0 + l;
      const int32_t *rec = k < n1 ? a.msgs + (beg1 + k) * kMsgFields : a.msgs2 + (beg2 + k - n1) * kMsgFields;
      const int4 *mp = reinterpret_cast<const int4 *>(rec);
      u = mp[0];
      v = mp[1];
    }
    const int T = u.x, S = u.y;
    const bool ok = l < cnt && T >= 1 && T <= 4 && (S == 1 || S == -1);
    const int code = !ok ? 0 : (T == 1 ? 1 : T == 4 ? 3 : 5) + (S == 1 ? 1 : 0);
    // times of valid messages must not decrease (R2): compare with the previous
    // valid lane, or with the last valid time before this chunk
    const uint64_t vmask = ballot(ok);
    if (vmask) {
      const uint64_t below = vmask & mask_lt();
      const int src = below ? 63 - __builtin_clzll(below) : 0;
      const int pts = from_lane(v.z, src), ptns = from_lane(v.w, src);
      const bool has_prev = below != 0 || st.seen;
      const int cts = below ? pts : st.last_ts, ctns = below ? ptns : st.last_tns;
      const bool dec = ok && has_prev && (v.z < cts || (v.z == cts && v.w < ctns));
      if (ballot(dec)) st.flags |= kFlagTimeOrder;
      const int top = 63 - __builtin_clzll(vmask);
      st.last_ts = rdlane(v.z, top);
      st.last_tns = rdlane(v.w, top);
      st.seen = 1;
    }
    st.n_msgs += cnt;
    for (int j = 0; j < cnt; ++j) {
      const int c = rdlane(code, j);
      process_msg(B, st, c, rdlane(u.z, j), rdlane(u.w, j), rdlane(v.x, j), rdlane(v.y, j), rdlane(v.z, j),
                  rdlane(v.w, j));
      if (l2_rows && k0 + j < n1) write_l2(B, st, a.levels, l2_rows + (k0 + j) * 4 * a.levels);
    }
  }
}

// Listed book i of a launch: its header and book from HBM, the first W slots of each
// side staged in LDS at `lds` (W = 0: none, every slot stays in HBM), its messages,
// then everything back.
template <bool SPILL>
__device__ void run_book(const ProcArgs &a, int i, int2 *lds, int W) {
  const int l = lane_id();
  const int book = a.book_ids ? uni(a.book_ids[i]) : i;
  if (book < 0 || book >= a.n_total) return;
  BookHdr *h = a.hdr + book;
  State st;
  st.n[0] = uni(h->n[0]);
  st.n[1] = uni(h->n[1]);
  st.cap = uni(h->cap);
  if (!SPILL && st.cap > W) {  // a book above the launch's capacity bound: left untouched
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
  const int row = a.out_rows ? uni(a.out_rows[i]) : i;  // output row of this book
  st.fills = a.fills ? a.fills + (int64_t)row * a.fill_cap * kTradeFields : nullptr;
  st.fill_cap = a.fill_cap;
  st.fill_count = 0;
  st.agent_tid = a.agent_tid;

  View<SPILL> B;
  B.lds = lds;
  B.hbm = a.books + uni64(h->book_off);
  B.W = W;
  B.cap = st.cap;

  // HBM -> LDS window
  for (int sd = 0; sd < 2; ++sd) {
    const int nw = st.n[sd] < W ? st.n[sd] : W;
    for (int p = 0; p < 3; ++p)
      for (int base = 0; base < nw; base += kWave)
        if (base + l < nw) lds[(sd * 3 + p) * W + base + l] = B.hbm[(int64_t)(sd * 3 + p) * st.cap + base + l];
  }
  load_best(B, st, 0);
  load_best(B, st, 1);

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
  if (a.prio_len > 0 && n1 >= a.prio_len) __builtin_amdgcn_s_setprio(3);
  // per-message L2 rows of source 1: contiguous by message index, or l2_stride
  // int32 apart per listed book
  int32_t *l2_rows = a.l2_mode != 1 ? nullptr
                     : a.l2_stride ? a.l2_out + (int64_t)i * a.l2_stride : a.l2_out + beg1 * 4 * a.levels;
  process_all(B, st, a, beg1, n1, (long long)i * a.w2, n2, l2_rows);
  if (a.l2_mode == 2) write_l2(B, st, a.levels, a.l2_out + (int64_t)row * 4 * a.levels);

  // LDS window -> HBM
  for (int sd = 0; sd < 2; ++sd) {
    const int nw = st.n[sd] < W ? st.n[sd] : W;
    for (int p = 0; p < 3; ++p)
      for (int base = 0; base < nw; base += kWave)
        if (base + l < nw) B.hbm[(int64_t)(sd * 3 + p) * st.cap + base + l] = lds[(sd * 3 + p) * W + base + l];
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

}  // namespace lds
}  // namespace lob
