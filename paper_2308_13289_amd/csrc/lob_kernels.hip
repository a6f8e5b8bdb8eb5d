// lob_kernels.hip -- gfx950 kernels of the batched limit-order-book matcher.
//
// One wavefront (64 lanes) owns one book for the whole of a call.  Each side of the
// book is kept SORTED in price-time priority (slot 0 = best) as three arrays of
// int2 pairs -- (P, Q), (OID, TID), (Ts, Tns) -- staged in LDS for the duration of
// the call.  Slot s of a side sits on lane s % 64 of chunk s / 64, so every book
// operation is a handful of wave-wide steps over the live chunks:
//   best standing order      slot 0 of the opposite side
//   matching loop            one inclusive prefix scan (DPP) of the crossing
//                            quantities: the fills are a prefix of the side, all of
//                            them full except possibly the last (Section 4.1)
//   add                      ballot-count of the orders ahead, shift the rest up
//   cancel / delete          ballot on OID (then on the initial-order rule of
//                            Section 5.1.1), shift the rest down if it empties
//   L2 top-k                 ballot of price changes + the same prefix scan
// The paper keeps unsorted arrays because under vmap every branch runs for every
// message and a sort would be paid each time (Section 4.3); here the eight
// (type x side) cases are a wave-uniform scalar branch, so only the work of the
// message at hand is done.
//
// Messages stream from HBM in 64-message chunks (one 32-byte record per lane) and
// are broadcast to scalar registers one at a time.  Trades go straight to the
// book's trade log as 24-byte records, one lane per fill, in fill order.
//
// Books whose capacity exceeds the LDS window W keep slots >= W in their HBM
// arrays (SPILL = true); the head of each side stays in LDS.
//
// Work distribution: one wave per listed book, workgroups dispatched in listed
// order.  For ragged batches the host lists books longest stream first, so the
// hardware workgroup dispatcher hands the next-longest book to whichever SIMD
// frees up first (longest-processing-time-first list scheduling).
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include "lob_device.h"
#include "lob_internal.h"

namespace lob {
namespace {

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
    const int incl = scan_incl(qv);
    const int excl = incl - qv;
    const bool takes = cross && excl < q;
    const uint64_t mt = ballot(takes);
    if (mt == 0) break;
    const int ntr = popc(mt);
    const bool full = cross && incl <= q;
    const int nfull = popc(ballot(full));
    int fill = 0;
    int2 ot = make_int2(0, 0);
    if (takes) {
      fill = min(qv, q - excl);
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

// Add (Section 4.1, item 1) on side SD: the new order goes behind every order with
// an equal or better price, i.e. at its price-time position.
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
  int pos = 0;
  // strictly better than the best order: it becomes slot 0, no search needed
  if (n > 0 && !(SD == 1 ? P > st.bP[SD] : P < st.bP[SD])) {
    for (int base = 0; base < n; base += kWave) {
      const int s = base + l;
      bool ahead = false;
      if (s < n) {
        const int p = B.at(SD, 0, s)->x;
        ahead = (SD == 1) ? p >= P : p <= P;
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
// out[0..L) as (price, qty); missing levels (-1, 0).  `scratch` holds L ints of LDS.
template <bool SPILL>
__device__ void l2_side(const View<SPILL> &B, const State &st, int sd, int L, int2 *out, int *scratch) {
  const int l = lane_id();
  const int n = st.n[sd];
  int lv_before = 0, q_before = 0, done = 0;
  for (int base = 0; base < n && done < L; base += kWave) {
    const int s = base + l;
    const bool valid = s < n;
    int2 pq = make_int2(0, 0);
    int prev = 0, next = 0;
    if (valid) {
      pq = *B.at(sd, 0, s);
      if (s > 0) prev = B.at(sd, 0, s - 1)->x;
      if (s + 1 < n) next = B.at(sd, 0, s + 1)->x;
    }
    const bool is_new = valid && (s == 0 || prev != pq.x);
    const bool is_last = valid && (s + 1 == n || next != pq.x);
    const int incl = q_before + scan_incl(valid ? pq.y : 0);
    const uint64_t mnew = ballot(is_new);
    const int lev = lv_before + popc(mnew & mask_le()) - 1;
    if (is_new && lev < L) scratch[lev] = incl - pq.y;
    if (is_last && lev < L) out[lev] = make_int2(pq.x, incl - scratch[lev]);
    lv_before += popc(mnew);
    done += popc(ballot(is_last));
    q_before = rdlane(incl, 63);
  }
  const int have = done < L ? done : L;
  if (l >= have && l < L) out[l] = make_int2(-1, 0);
}

template <bool SPILL>
__device__ __forceinline__ void write_l2(const View<SPILL> &B, const State &st, int L, int32_t *row,
                                         int *scratch) {
  int2 *o = reinterpret_cast<int2 *>(row);
  l2_side(B, st, 0, L, o, scratch);
  l2_side(B, st, 1, L, o + L, scratch);
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
                                            long long n1, long long beg2, long long n2, int32_t *l2_rows,
                                            int *scratch) {
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
      if (l2_rows && k0 + j < n1) write_l2(B, st, a.levels, l2_rows + (k0 + j) * 4 * a.levels, scratch);
    }
  }
}

template <bool SPILL>
__device__ void run_book(const ProcArgs &a, int i, int2 *lds, int *scratch) {
  const int l = lane_id();
  const int book = a.book_ids ? uni(a.book_ids[i]) : i;
  if (book < 0 || book >= a.n_total) return;
  BookHdr *h = a.hdr + book;
  State st;
  st.n[0] = uni(h->n[0]);
  st.n[1] = uni(h->n[1]);
  st.cap = uni(h->cap);
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
  B.W = a.W;
  B.cap = st.cap;

  // HBM -> LDS window
  for (int sd = 0; sd < 2; ++sd) {
    const int nw = st.n[sd] < a.W ? st.n[sd] : a.W;
    for (int p = 0; p < 3; ++p)
      for (int base = 0; base < nw; base += kWave)
        if (base + l < nw) lds[(sd * 3 + p) * a.W + base + l] = B.hbm[(int64_t)(sd * 3 + p) * st.cap + base + l];
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
  process_all(B, st, a, beg1, n1, (long long)i * a.w2, n2, l2_rows, scratch);
  if (a.l2_mode == 2) write_l2(B, st, a.levels, a.l2_out + (int64_t)row * 4 * a.levels, scratch);

  // LDS window -> HBM
  for (int sd = 0; sd < 2; ++sd) {
    const int nw = st.n[sd] < a.W ? st.n[sd] : a.W;
    for (int p = 0; p < 3; ++p)
      for (int base = 0; base < nw; base += kWave)
        if (base + l < nw) B.hbm[(int64_t)(sd * 3 + p) * st.cap + base + l] = lds[(sd * 3 + p) * a.W + base + l];
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

template <bool SPILL>
__global__ void __launch_bounds__(1024) k_process(ProcArgs a) {
  extern __shared__ int2 smem[];
  const int w = uni(threadIdx.x / kWave);  // uniform: one wave = one book
  const int i = blockIdx.x * a.bpb + w;
  if (i >= a.n) return;
  int2 *lds = smem + (int64_t)w * a.lds_int2_per_wave;
  int *scratch = reinterpret_cast<int *>(lds + 6 * a.W);
  run_book<SPILL>(a, i, lds, scratch);
}

// ---------------------------------------------------------------- small kernels

__global__ void k_reset(BookHdr *hdr, const int32_t *ids, int n, int n_total) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = ids ? ids[i] : i;
  if (b < 0 || b >= n_total) return;
  BookHdr *h = hdr + b;
  h->n[0] = h->n[1] = 0;
  h->flags = 0;
  h->log_count = 0;
  h->n_msgs = h->n_trades = h->limit_qty = h->market_qty = h->traded_qty = h->cancelled_qty = 0;
  h->market_discarded = h->rejected_qty = h->cancel_miss = 0;
  h->last_ts = h->last_tns = 0;
  h->seen_time = 0;
}

struct StatusOut {
  int64_t n_msgs, n_trades, limit_qty, market_qty, traded_qty, cancelled_qty, market_discarded,
      rejected_qty, cancel_miss;
  int32_t flags, n_ask, n_bid, pad;
  int64_t log_records;
};

__global__ void k_status(const BookHdr *hdr, const int32_t *ids, int n, int n_total, StatusOut *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = ids ? ids[i] : i;
  StatusOut o;
  if (b < 0 || b >= n_total) {
    memset(&o, 0, sizeof(o));
    o.flags = -1;
    out[i] = o;
    return;
  }
  const BookHdr *h = hdr + b;
  o.n_msgs = h->n_msgs;
  o.n_trades = h->n_trades;
  o.limit_qty = h->limit_qty;
  o.market_qty = h->market_qty;
  o.traded_qty = h->traded_qty;
  o.cancelled_qty = h->cancelled_qty;
  o.market_discarded = h->market_discarded;
  o.rejected_qty = h->rejected_qty;
  o.cancel_miss = h->cancel_miss;
  o.flags = h->flags;
  o.n_ask = h->n[0];
  o.n_bid = h->n[1];
  o.pad = 0;
  o.log_records = h->log_count;
  out[i] = o;
}

// L2 straight from the HBM arrays: one wave per listed book, W = 0.
__global__ void __launch_bounds__(256) k_read_l2(const BookHdr *hdr, int2 *books, const int32_t *ids, int n,
                                                  int n_total, int L, int32_t *out) {
  __shared__ int scratch_all[4 * 64];
  const int w = uni(threadIdx.x / kWave);  // uniform: one wave = one book
  const int i = blockIdx.x * 4 + w;
  if (i >= n) return;
  const int b = ids ? uni(ids[i]) : i;
  if (b < 0 || b >= n_total) return;
  const BookHdr *h = hdr + b;
  View<true> B;
  B.lds = nullptr;
  B.hbm = books + h->book_off;
  B.W = 0;
  B.cap = uni(h->cap);
  State st;
  st.n[0] = uni(h->n[0]);
  st.n[1] = uni(h->n[1]);
  write_l2(B, st, L, out + (int64_t)i * 4 * L, scratch_all + w * 64);
}

// Book dump [n][2][dump_cap][6]: one wave per listed book.
__global__ void __launch_bounds__(256) k_read_book(const BookHdr *hdr, const int2 *books, const int32_t *ids,
                                                    int n, int n_total, int dump_cap, int32_t *out) {
  const int w = uni(threadIdx.x / kWave);  // uniform: one wave = one book
  const int i = blockIdx.x * 4 + w;
  if (i >= n) return;
  const int l = lane_id();
  const int bid = ids ? uni(ids[i]) : i;
  if (bid < 0 || bid >= n_total) return;
  const BookHdr *h = hdr + bid;
  const int cap = h->cap;
  const int2 *bk = books + h->book_off;
  for (int sd = 0; sd < 2; ++sd) {
    const int live = h->n[sd];
    int32_t *o = out + ((int64_t)i * 2 + sd) * dump_cap * 6;
    for (int base = 0; base < dump_cap; base += kWave) {
      const int s = base + l;
      if (s >= dump_cap) continue;
      int2 a = make_int2(-1, -1), b = a, c = a;
      if (s < live) {
        a = bk[(sd * 3 + 0) * cap + s];
        b = bk[(sd * 3 + 1) * cap + s];
        c = bk[(sd * 3 + 2) * cap + s];
      }
      int32_t *r = o + (int64_t)s * 6;
      r[0] = a.x; r[1] = a.y; r[2] = b.x; r[3] = b.y; r[4] = c.x; r[5] = c.y;
    }
  }
}

// Load a book dump: rows taken in order up to the first with Q <= 0 or the capacity.
__global__ void __launch_bounds__(256) k_write_book(BookHdr *hdr, int2 *books, const int32_t *ids, int n,
                                                     int n_total, int dump_cap, const int32_t *in) {
  const int w = uni(threadIdx.x / kWave);  // uniform: one wave = one book
  const int i = blockIdx.x * 4 + w;
  if (i >= n) return;
  const int l = lane_id();
  const int bid = ids ? uni(ids[i]) : i;
  if (bid < 0 || bid >= n_total) return;
  BookHdr *h = hdr + bid;
  const int cap = uni(h->cap);
  int2 *bk = books + h->book_off;
  int bad = 0;
  for (int sd = 0; sd < 2; ++sd) {
    const int32_t *src = in + ((int64_t)i * 2 + sd) * dump_cap * 6;
    const int lim = dump_cap < cap ? dump_cap : cap;
    int live = lim;
    for (int base = 0; base < lim; base += kWave) {
      const int s = base + l;
      const bool stop = s < lim && src[(int64_t)s * 6 + 1] <= 0;
      const uint64_t m = ballot(stop);
      if (m) {
        live = base + first_set(m);
        break;
      }
    }
    if (live == cap && dump_cap > cap && src[(int64_t)cap * 6 + 1] > 0) bad = 1;
    for (int base = 0; base < live; base += kWave) {
      const int s = base + l;
      bool unsorted = false;
      if (s < live) {
        const int32_t *r = src + (int64_t)s * 6;
        bk[(sd * 3 + 0) * cap + s] = make_int2(r[0], r[1]);
        bk[(sd * 3 + 1) * cap + s] = make_int2(r[2], r[3]);
        bk[(sd * 3 + 2) * cap + s] = make_int2(r[4], r[5]);
        if (s > 0) unsorted = sd == 0 ? r[0] < r[-6] : r[0] > r[-6];
      }
      if (ballot(unsorted)) bad = 1;
    }
    if (l == 0) h->n[sd] = live;
  }
  if (l == 0 && bad) h->flags |= kFlagBadLoad;
}

// Book initialisation from an L2 snapshot (Section 5.1.1): one wave per book, lane
// l holds level l of both sides.  The book is emptied with its counters and log;
// a snapshot that is a book (strictly ordered prices, not crossed, fits the
// capacity) becomes one order per present level (qty > 0), ids -9000, -9001, ...
// level by level with the ask before the bid; otherwise the book stays empty and
// is flagged.
__global__ void __launch_bounds__(256) k_seed_l2(BookHdr *hdr, int2 *books, const int32_t *ids, int n,
                                                  int n_total, int L, const int32_t *l2, const int32_t *times,
                                                  int tid) {
  const int w = uni(threadIdx.x / kWave);  // uniform: one wave = one book
  const int i = blockIdx.x * 4 + w;
  if (i >= n) return;
  const int l = lane_id();
  const int bid = ids ? uni(ids[i]) : i;
  if (bid < 0 || bid >= n_total) return;
  BookHdr *h = hdr + bid;
  const int cap = uni(h->cap);
  int2 *bk = books + uni64(h->book_off);
  const int2 *row = reinterpret_cast<const int2 *>(l2) + (int64_t)i * 2 * L;  // [2][L] (price, qty)
  int2 e[2];
  uint64_t mp[2];
  int cnt[2], best[2];
  bool bad = false;
  for (int sd = 0; sd < 2; ++sd) {
    e[sd] = l < L ? row[sd * L + l] : make_int2(0, 0);
    const bool pres = (l < L) & (e[sd].y > 0);
    mp[sd] = ballot(pres);
    cnt[sd] = popc(mp[sd]);
    // strictly ordered: each present level against the previous present one
    const uint64_t below = mp[sd] & mask_lt();
    const int src = below ? 63 - __builtin_clzll(below) : 0;
    const int prev = from_lane(e[sd].x, src);
    const bool unordered = pres & (below != 0) & (sd == 0 ? e[sd].x <= prev : e[sd].x >= prev);
    if (ballot(unordered) || cnt[sd] > cap) bad = true;
    best[sd] = mp[sd] ? rdlane(e[sd].x, first_set(mp[sd])) : 0;
  }
  if (cnt[0] > 0 && cnt[1] > 0 && best[1] >= best[0]) bad = true;
  const int ts = times ? uni(times[2 * i]) : 0, tns = times ? uni(times[2 * i + 1]) : 0;
  if (!bad) {
    // rank in the order ask 0, bid 0, ask 1, bid 1, ...
    const int before = popc(mp[0] & mask_lt()) + popc(mp[1] & mask_lt());
    for (int sd = 0; sd < 2; ++sd) {
      const bool pres = (mp[sd] >> l) & 1;
      if (pres) {
        const int slot = popc(mp[sd] & mask_lt());
        const int oid = -9000 - before - (sd == 1 && ((mp[0] >> l) & 1) ? 1 : 0);
        bk[(sd * 3 + 0) * cap + slot] = make_int2(e[sd].x, e[sd].y);
        bk[(sd * 3 + 1) * cap + slot] = make_int2(oid, tid);
        bk[(sd * 3 + 2) * cap + slot] = make_int2(ts, tns);
      }
    }
  }
  if (l == 0) {
    h->n[0] = bad ? 0 : cnt[0];
    h->n[1] = bad ? 0 : cnt[1];
    h->flags = bad ? kFlagBadLoad : 0;
    h->log_count = 0;
    h->n_msgs = h->n_trades = h->limit_qty = h->market_qty = h->traded_qty = h->cancelled_qty = 0;
    h->market_discarded = h->rejected_qty = h->cancel_miss = 0;
    h->last_ts = h->last_tns = 0;
    h->seen_time = 0;
  }
}

// Trade-log drain, pass 1 (one block): counts and exclusive offsets.
__global__ void __launch_bounds__(1024) k_trade_counts(const BookHdr *hdr, const int32_t *ids, int n,
                                                        int n_total, int64_t *counts, int64_t *offsets) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int b = t * per, e = min(n, b + per);
  int64_t sum = 0;
  for (int i = b; i < e; ++i) {
    const int bid = ids ? ids[i] : i;
    const int64_t c = (bid >= 0 && bid < n_total) ? hdr[bid].log_count : 0;
    counts[i] = c;
    sum += c;
  }
  part[t] = sum;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int64_t v = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - sum;
  for (int i = b; i < e; ++i) {
    offsets[i] = run;
    run += counts[i];
  }
  if (t == 1023) offsets[n] = part[1023];
}

// Pass 2 (one block per listed book): copy the records that fit and empty the log.
__global__ void __launch_bounds__(256) k_trade_copy(BookHdr *hdr, const int32_t *log, const int32_t *ids,
                                                     int n, int n_total, const int64_t *counts,
                                                     const int64_t *offsets, int64_t max_records, int32_t *out) {
  const int i = blockIdx.x;
  if (i >= n) return;
  if (offsets[i + 1] > max_records) return;
  const int bid = ids ? ids[i] : i;
  if (bid < 0 || bid >= n_total) return;
  BookHdr *h = hdr + bid;
  const int64_t cnt = counts[i];
  const int2 *src = reinterpret_cast<const int2 *>(log + h->log_off * kTradeFields);
  int2 *dst = reinterpret_cast<int2 *>(out + offsets[i] * kTradeFields);
  for (int64_t k = threadIdx.x; k < cnt * 3; k += blockDim.x) dst[k] = src[k];
  __syncthreads();
  if (threadIdx.x == 0) h->log_count = 0;
}

__global__ void k_selftest(int32_t *out) {
  // lanes: scan of (lane % 7 + 1), ballot/mask checks
  const int l = lane_id();
  const int v = l % 7 + 1;
  out[l] = scan_incl(v);
  out[64 + l] = popc(ballot(l % 3 == 0) & mask_le());
  out[128 + l] = popc(mask_lt());
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_process(const ProcArgs &a, bool spill, hipStream_t s) {
  const int threads = a.bpb * kWave;
  const size_t lds = (size_t)a.bpb * a.lds_int2_per_wave * sizeof(int2);
  const int grid = (a.n + a.bpb - 1) / a.bpb;
  if (spill)
    hipLaunchKernelGGL(k_process<true>, dim3(grid), dim3(threads), lds, s, a);
  else
    hipLaunchKernelGGL(k_process<false>, dim3(grid), dim3(threads), lds, s, a);
  return hipGetLastError();
}

hipError_t set_process_lds_limit(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void *)k_process<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)k_process<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

hipError_t launch_reset(BookHdr *hdr, const int32_t *ids, int n, int n_total, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3((n + 255) / 256), dim3(256), 0, s, hdr, ids, n, n_total);
  return hipGetLastError();
}

hipError_t launch_status(const BookHdr *hdr, const int32_t *ids, int n, int n_total, void *out, hipStream_t s) {
  hipLaunchKernelGGL(k_status, dim3((n + 255) / 256), dim3(256), 0, s, hdr, ids, n, n_total,
                     reinterpret_cast<StatusOut *>(out));
  return hipGetLastError();
}

hipError_t launch_read_l2(const BookHdr *hdr, int2 *books, const int32_t *ids, int n, int n_total, int L,
                          int32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_read_l2, dim3((n + 3) / 4), dim3(256), 0, s, hdr, books, ids, n, n_total, L, out);
  return hipGetLastError();
}

hipError_t launch_read_book(const BookHdr *hdr, const int2 *books, const int32_t *ids, int n, int n_total,
                            int dump_cap, int32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_read_book, dim3((n + 3) / 4), dim3(256), 0, s, hdr, books, ids, n, n_total, dump_cap,
                     out);
  return hipGetLastError();
}

hipError_t launch_write_book(BookHdr *hdr, int2 *books, const int32_t *ids, int n, int n_total, int dump_cap,
                             const int32_t *in, hipStream_t s) {
  hipLaunchKernelGGL(k_write_book, dim3((n + 3) / 4), dim3(256), 0, s, hdr, books, ids, n, n_total, dump_cap,
                     in);
  return hipGetLastError();
}

hipError_t launch_read_trades(BookHdr *hdr, const int32_t *log, const int32_t *ids, int n, int n_total,
                              int32_t *out, int64_t max_records, int64_t *counts, int64_t *offsets,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_trade_counts, dim3(1), dim3(1024), 0, s, hdr, ids, n, n_total, counts, offsets);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n == 0) return e;
  hipLaunchKernelGGL(k_trade_copy, dim3(n), dim3(256), 0, s, hdr, log, ids, n, n_total, counts, offsets,
                     max_records, out);
  return hipGetLastError();
}

hipError_t launch_seed_l2(BookHdr *hdr, int2 *books, const int32_t *ids, int n, int n_total, int L,
                          const int32_t *l2, const int32_t *times, int tid, hipStream_t s) {
  hipLaunchKernelGGL(k_seed_l2, dim3((n + 3) / 4), dim3(256), 0, s, hdr, books, ids, n, n_total, L, l2, times, tid);
  return hipGetLastError();
}

hipError_t launch_selftest(int32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_selftest, dim3(1), dim3(64), 0, s, out);
  return hipGetLastError();
}

}  // namespace lob
