// lob_regbook.hip -- matching kernel with the top of each book side in registers.
//
// Same algorithm and results as lob_kernels.hip (one wavefront per book, each side
// kept in price-time priority, slot 0 = best), different residency: slots
// [0, 128) of each side live in VGPRs as two 64-lane chunks (slot 64c + lane in
// chunk c), slots [128, W) in the LDS window and slots [W, capacity) in HBM.  A
// book that never holds more than 128 orders on a side therefore never touches
// LDS or HBM for its orders while it runs: the best order is lane 0 of chunk 0,
// moving orders by one slot is a DPP wave shift (wave_shr:1 / wave_shl:1) with the
// neighbouring chunk's edge lane carried in, and moving them by more than one
// slot is a ds_bpermute.  The eight (type x side) message cases of the paper
// (Section 4.2) are compile-time specialisations behind one wave-uniform branch.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include "lob_device.h"
#include "lob_internal.h"

namespace lob {
namespace {

using namespace dev;

constexpr int R = 2;            // register chunks per side
constexpr int RS = R * kWave;   // slots per side held in registers

// One 64-slot chunk of a side: (P, Q), (OID, TID), (Ts, Tns) of slot 64c + lane.
struct Chunk {
  int2 pq, ot, tt;
};

__device__ __forceinline__ Chunk zero_chunk() {
  Chunk z;
  z.pq = z.ot = z.tt = make_int2(0, 0);
  return z;
}

__device__ __forceinline__ Chunk lane_of(const Chunk &x, int l) {  // uniform value of lane l
  Chunk v;
  v.pq = make_int2(rdlane(x.pq.x, l), rdlane(x.pq.y, l));
  v.ot = make_int2(rdlane(x.ot.x, l), rdlane(x.ot.y, l));
  v.tt = make_int2(rdlane(x.tt.x, l), rdlane(x.tt.y, l));
  return v;
}

__device__ __forceinline__ Chunk shr1c(const Chunk &x, const Chunk &fill) {
  Chunk v;
  v.pq = make_int2(shr1(x.pq.x, fill.pq.x), shr1(x.pq.y, fill.pq.y));
  v.ot = make_int2(shr1(x.ot.x, fill.ot.x), shr1(x.ot.y, fill.ot.y));
  v.tt = make_int2(shr1(x.tt.x, fill.tt.x), shr1(x.tt.y, fill.tt.y));
  return v;
}

__device__ __forceinline__ Chunk shl1c(const Chunk &x, const Chunk &fill) {
  Chunk v;
  v.pq = make_int2(shl1(x.pq.x, fill.pq.x), shl1(x.pq.y, fill.pq.y));
  v.ot = make_int2(shl1(x.ot.x, fill.ot.x), shl1(x.ot.y, fill.ot.y));
  v.tt = make_int2(shl1(x.tt.x, fill.tt.x), shl1(x.tt.y, fill.tt.y));
  return v;
}

__device__ __forceinline__ Chunk from_lane_c(const Chunk &x, int src) {
  Chunk v;
  v.pq = make_int2(from_lane(x.pq.x, src), from_lane(x.pq.y, src));
  v.ot = make_int2(from_lane(x.ot.x, src), from_lane(x.ot.y, src));
  v.tt = make_int2(from_lane(x.tt.x, src), from_lane(x.tt.y, src));
  return v;
}

__device__ __forceinline__ Chunk pick(bool c, const Chunk &a, const Chunk &b) {
  Chunk v;
  v.pq = c ? a.pq : b.pq;
  v.ot = c ? a.ot : b.ot;
  v.tt = c ? a.tt : b.tt;
  return v;
}

template <bool SPILL>
struct Book {
  Chunk r[2][R];  // [side][chunk], indexed with compile-time constants only
  int2 *lds;      // [2][3][W - RS] window for slots [RS, W)
  int2 *hbm;      // [2][3][cap] the book's arrays
  int W, cap;
  __device__ __forceinline__ int2 *tail(int sd, int p, int s) const {  // s >= RS
    const int tw = W - RS;
    if constexpr (!SPILL) {
      return lds + (sd * 3 + p) * tw + (s - RS);
    } else {
      return s < W ? lds + (sd * 3 + p) * tw + (s - RS) : hbm + (int64_t)(sd * 3 + p) * cap + s;
    }
  }
  __device__ __forceinline__ Chunk tail_read(int sd, int s) const {
    Chunk v;
    v.pq = *tail(sd, 0, s);
    v.ot = *tail(sd, 1, s);
    v.tt = *tail(sd, 2, s);
    return v;
  }
  __device__ __forceinline__ void tail_write(int sd, int s, const Chunk &v) const {
    *tail(sd, 0, s) = v.pq;
    *tail(sd, 1, s) = v.ot;
    *tail(sd, 2, s) = v.tt;
  }
};

template <bool SPILL>
__device__ __forceinline__ void fence_tail() {
  if constexpr (SPILL) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// uniform (P, Q) of slot k of side SD
template <int SD, bool SPILL>
__device__ __forceinline__ int2 slot_pq(const Book<SPILL> &B, int k) {
  if (k >= RS) {
    const int2 v = *B.tail(SD, 0, k);
    return make_int2(uni(v.x), uni(v.y));
  }
  int2 v = make_int2(0, 0);
#pragma unroll
  for (int c = 0; c < R; ++c)
    if ((k >> 6) == c) v = make_int2(rdlane(B.r[SD][c].pq.x, k & 63), rdlane(B.r[SD][c].pq.y, k & 63));
  return v;
}

// Slots [from+m, n) of side SD move to [from, n-m).
template <int SD, bool SPILL>
__device__ __forceinline__ void shift_down_r(Book<SPILL> &B, int from, int m, int n) {
  const int l = lane_id_local();
  Chunk nw[R];
  if (m == 1) {
#pragma unroll
    for (int c = 0; c < R; ++c) {
      Chunk carry = zero_chunk();  // slot 64(c+1)
      if (c + 1 < R)
        carry = lane_of(B.r[SD][c + 1], 0);
      else if (RS < n) {
        carry = B.tail_read(SD, RS);
        carry.pq = make_int2(uni(carry.pq.x), uni(carry.pq.y));
        carry.ot = make_int2(uni(carry.ot.x), uni(carry.ot.y));
        carry.tt = make_int2(uni(carry.tt.x), uni(carry.tt.y));
      }
      nw[c] = shl1c(B.r[SD][c], carry);
    }
  } else {
    const int q = m >> 6, rr = m & 63;
    const int src_lane = (l + rr) & 63;
    const bool low = (l + rr) < 64;
#pragma unroll
    for (int c = 0; c < R; ++c) {
      Chunk v0 = zero_chunk(), v1 = zero_chunk();
#pragma unroll
      for (int k = 0; k < R; ++k) {
        if (c + q == k) v0 = from_lane_c(B.r[SD][k], src_lane);
        if (c + q + 1 == k) v1 = from_lane_c(B.r[SD][k], src_lane);
      }
      Chunk v = pick(low, v0, v1);
      const int src = c * kWave + l + m;
      if (src >= RS && src < n) v = B.tail_read(SD, src);
      nw[c] = v;
    }
  }
  fence_tail<SPILL>();
  // the tail moves down; its sources are all tail slots
  const int t0 = from > RS ? from : RS;
  for (int base = t0 & ~63; base < n - m; base += kWave) {
    const int s = base + lane_id_local();
    const bool act = s >= t0 && s < n - m;
    Chunk v;
    if (act) v = B.tail_read(SD, s + m);
    if (act) B.tail_write(SD, s, v);
    fence_tail<SPILL>();
  }
#pragma unroll
  for (int c = 0; c < R; ++c) {
    const int s = c * kWave + l;
    if (s >= from && s < n - m) B.r[SD][c] = nw[c];
  }
}

// Slots [pos, n) of side SD move to [pos+1, n+1).  Requires n < capacity.
template <int SD, bool SPILL>
__device__ __forceinline__ void shift_up_r(Book<SPILL> &B, int pos, int n) {
  const int l = lane_id_local();
  // the tail first, top down
  if (n > RS) {
    const int t0 = pos > RS ? pos : RS;
    for (int base = (n - 1) & ~63; base >= (t0 & ~63); base -= kWave) {
      const int s = base + lane_id_local();
      const bool act = s >= t0 && s < n;
      Chunk v;
      if (act) v = B.tail_read(SD, s);
      if (act) B.tail_write(SD, s + 1, v);
      fence_tail<SPILL>();
    }
  }
  // the last register slot crosses into the tail
  if (n >= RS && pos <= RS - 1) {
    const Chunk v = lane_of(B.r[SD][R - 1], 63);
    if (l == 0) B.tail_write(SD, RS, v);
    fence_tail<SPILL>();
  }
  // registers, top chunk first (each chunk takes its lower neighbour's lane 63)
#pragma unroll
  for (int c = R - 1; c >= 0; --c) {
    if (c * kWave + 63 > pos && c * kWave <= n) {
      Chunk carry = zero_chunk();
      if (c > 0) carry = lane_of(B.r[SD][c - 1], 63);
      const Chunk sh = shr1c(B.r[SD][c], carry);
      const int s = c * kWave + l;
      if (s > pos && s <= n) B.r[SD][c] = sh;
    }
  }
}

// Matching loop of Section 4.1 against side OPP; returns the unfilled quantity.
template <int OPP, bool SPILL>
__device__ __forceinline__ int match_r(Book<SPILL> &B, State &st, int lim, int q, int a_oid, int a_tid, int ts, int tns) {
  const int l = lane_id_local();
  const int n = st.n[OPP];
  constexpr bool buyer = (OPP == 0);
  int removed = 0;
  bool more = true;  // every order seen so far was filled completely
#pragma unroll
  for (int c = 0; c < R; ++c) {
    if (more && c * kWave < n && q > 0) {
      Chunk &x = B.r[OPP][c];
      const int s = c * kWave + l;
      const bool valid = s < n;
      const bool cross = valid && (buyer ? x.pq.x <= lim : x.pq.x >= lim);
      const int qv = cross ? x.pq.y : 0;
      const int incl = scan_incl(qv);
      const int excl = incl - qv;
      const bool takes = cross && excl < q;
      const uint64_t mt = ballot(takes);
      if (mt == 0) {
        more = false;
      } else {
        const int ntr = popc(mt);
        const bool full = cross && incl <= q;
        const int nfull = popc(ballot(full));
        const int fill = takes ? min(qv, q - excl) : 0;
        emit(st, takes, ntr, x.pq.x, fill, x.ot.x, a_oid, ts, tns, x.ot.y, a_tid);
        if (takes && !full) x.pq.y -= fill;
        const int consumed = (nfull == ntr) ? rdlane(incl, ntr - 1) : q;
        st.traded_qty += consumed;
        st.n_trades += ntr;
        q -= consumed;
        removed += nfull;
        if (nfull < kWave) more = false;
      }
    } else {
      more = false;
    }
  }
  if (more && q > 0) {
    for (int base = RS; base < n && q > 0; base += kWave) {
      const int s = base + lane_id_local();
      const bool valid = s < n;
      int2 pq = make_int2(0, 0);
      if (valid) pq = *B.tail(OPP, 0, s);
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
        ot = *B.tail(OPP, 1, s);
        if (!full) *B.tail(OPP, 0, s) = make_int2(pq.x, pq.y - fill);
      }
      emit(st, takes, ntr, pq.x, fill, ot.x, a_oid, ts, tns, ot.y, a_tid);
      const int consumed = (nfull == ntr) ? rdlane(incl, ntr - 1) : q;
      st.traded_qty += consumed;
      st.n_trades += ntr;
      q -= consumed;
      removed += nfull;
      if (nfull < kWave) break;
    }
    fence_tail<SPILL>();
  }
  if (removed > 0) {
    shift_down_r<OPP>(B, 0, removed, n);
    st.n[OPP] = n - removed;
  }
  return q;
}

// Add (Section 4.1, item 1) at the order's price-time position on side SD.
template <int SD, bool SPILL>
__device__ __forceinline__ void insert_r(Book<SPILL> &B, State &st, int P, int Q, int oid, int tid, int ts, int tns) {
  const int l = lane_id_local();
  const int n = st.n[SD];
  if (n >= st.cap) {
    st.rejected_qty += Q;
    st.flags |= kFlagSideFull;
    return;
  }
  int pos = 0;
  bool more = true;
#pragma unroll
  for (int c = 0; c < R; ++c) {
    if (more && c * kWave < n) {
      const int s = c * kWave + l;
      const int p = B.r[SD][c].pq.x;
      const bool ahead = s < n && (SD == 1 ? p >= P : p <= P);
      const int k = popc(ballot(ahead));
      pos += k;
      if (k < kWave) more = false;
    } else {
      more = false;
    }
  }
  if (more) {
    for (int base = RS; base < n; base += kWave) {
      const int s = base + lane_id_local();
      bool ahead = false;
      if (s < n) {
        const int p = B.tail(SD, 0, s)->x;
        ahead = SD == 1 ? p >= P : p <= P;
      }
      const int k = popc(ballot(ahead));
      pos += k;
      if (k < kWave) break;
    }
  }
  if (pos < n) shift_up_r<SD>(B, pos, n);
  Chunk o;
  o.pq = make_int2(P, Q);
  o.ot = make_int2(oid, tid);
  o.tt = make_int2(ts, tns);
  if (pos < RS) {
#pragma unroll
    for (int c = 0; c < R; ++c)
      if ((pos >> 6) == c && l == (pos & 63)) B.r[SD][c] = o;
  } else {
    if (l == 0) B.tail_write(SD, pos, o);
    fence_tail<SPILL>();
  }
  st.n[SD] = n + 1;
}

// first slot of side SD (registers, then tail) where the predicate holds, or -1
template <int SD, bool SPILL, bool FALLBACK>
__device__ __forceinline__ int find_r(const Book<SPILL> &B, int n, int oid, int price) {
  const int l = lane_id_local();
#pragma unroll
  for (int c = 0; c < R; ++c) {
    if (c * kWave < n) {
      const Chunk &x = B.r[SD][c];
      const int s = c * kWave + l;
      const bool hit = s < n && (FALLBACK ? (x.ot.x <= -9000 && x.pq.x == price) : x.ot.x == oid);
      const uint64_t m = ballot(hit);
      if (m) return c * kWave + first_set(m);
    }
  }
  for (int base = RS; base < n; base += kWave) {
    const int s = base + lane_id_local();
    bool hit = false;
    if (s < n) {
      const int o = B.tail(SD, 1, s)->x;
      hit = FALLBACK ? (o <= -9000 && B.tail(SD, 0, s)->x == price) : o == oid;
    }
    const uint64_t m = ballot(hit);
    if (m) return base + first_set(m);
  }
  return -1;
}

// Cancel / delete (Section 4.1, item 2; Section 5.1.1 for initial orders).
template <int SD, bool SPILL>
__device__ __forceinline__ void cancel_r(Book<SPILL> &B, State &st, int oid, int qty, int price) {
  if (qty <= 0) return;
  const int l = lane_id_local();
  const int n = st.n[SD];
  int k = find_r<SD, SPILL, false>(B, n, oid, price);
  if (k < 0) k = find_r<SD, SPILL, true>(B, n, oid, price);
  if (k < 0) {
    st.cancel_miss++;
    return;
  }
  const int2 pq = slot_pq<SD>(B, k);
  st.cancelled_qty += min(qty, pq.y);
  const int left = pq.y - qty;
  if (left > 0) {
    if (k < RS) {
#pragma unroll
      for (int c = 0; c < R; ++c)
        if ((k >> 6) == c && l == (k & 63)) B.r[SD][c].pq.y = left;
    } else {
      if (l == 0) *B.tail(SD, 0, k) = make_int2(pq.x, left);
      fence_tail<SPILL>();
    }
  } else {
    shift_down_r<SD>(B, k, 1, n);
    st.n[SD] = n - 1;
  }
}

// L2 of side SD into out[0..L) (price, summed qty); missing levels (-1, 0).
template <int SD, bool SPILL>
__device__ __forceinline__ void l2_side_r(const Book<SPILL> &B, const State &st, int L, int2 *out, int *scratch) {
  const int l = lane_id_local();
  const int n = st.n[SD];
  int lv_before = 0, q_before = 0, done = 0;
#pragma unroll
  for (int c = 0; c < R; ++c) {
    if (c * kWave < n && done < L) {
      const Chunk &x = B.r[SD][c];
      const int s = c * kWave + l;
      const bool valid = s < n;
      const int prev_fill = c > 0 ? rdlane(B.r[SD][c - 1].pq.x, 63) : 0;
      int next_fill = 0;
      if (c + 1 < R)
        next_fill = rdlane(B.r[SD][c + 1].pq.x, 0);
      else if (RS < n)
        next_fill = uni(B.tail(SD, 0, RS)->x);
      const int prev = shr1(x.pq.x, prev_fill);
      const int next = shl1(x.pq.x, next_fill);
      const bool is_new = valid && (s == 0 || prev != x.pq.x);
      const bool is_last = valid && (s + 1 == n || next != x.pq.x);
      const int incl = q_before + scan_incl(valid ? x.pq.y : 0);
      const uint64_t mnew = ballot(is_new);
      const int lev = lv_before + popc(mnew & mask_le()) - 1;
      if (is_new && lev < L) scratch[lev] = incl - x.pq.y;
      if (is_last && lev < L) out[lev] = make_int2(x.pq.x, incl - scratch[lev]);
      lv_before += popc(mnew);
      done += popc(ballot(is_last));
      q_before = rdlane(incl, 63);
    }
  }
  for (int base = RS; base < n && done < L; base += kWave) {
    const int s = base + lane_id_local();
    const bool valid = s < n;
    int2 pq = make_int2(0, 0);
    int prev = 0, next = 0;
    const int edge = rdlane(B.r[SD][R - 1].pq.x, 63);  // slot RS-1
    if (valid) {
      pq = *B.tail(SD, 0, s);
      prev = s == RS ? edge : B.tail(SD, 0, s - 1)->x;
      if (s + 1 < n) next = B.tail(SD, 0, s + 1)->x;
    }
    const bool is_new = valid && prev != pq.x;
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
__device__ __forceinline__ void write_l2_r(const Book<SPILL> &B, const State &st, int L, int32_t *row,
                                           int *scratch) {
  int2 *o = reinterpret_cast<int2 *>(row);
  l2_side_r<0>(B, st, L, o, scratch);
  l2_side_r<1>(B, st, L, o + L, scratch);
}

// One message (Section 4.2): the eight (type x side) cases.
template <bool SPILL>
__device__ __forceinline__ void process_msg_r(Book<SPILL> &B, State &st, int T, int S, int P, int Q, int oid,
                                              int tid, int ts, int tns) {
  st.n_msgs++;
  if (T < 1 || T > 4 || (S != 1 && S != -1)) return;
  if (st.seen && (ts < st.last_ts || (ts == st.last_ts && tns < st.last_tns))) st.flags |= kFlagTimeOrder;
  st.seen = 1;
  st.last_ts = ts;
  st.last_tns = tns;
  if (T == 1 || T == 4) {
    // limit: match, then rest the remainder (Section 4.2, item 1); market: match at
    // price 0 (sell) or max_int (buy), drop the remainder (item 3)
    if (Q > 0) {
      if (T == 1)
        st.limit_qty += Q;
      else
        st.market_qty += Q;
    }
    const int lim = T == 1 ? P : (S == 1 ? INT_MAX : 0);
    const int rem = S == 1 ? match_r<0>(B, st, lim, Q, oid, tid, ts, tns) : match_r<1>(B, st, lim, Q, oid, tid, ts, tns);
    if (rem > 0) {
      if (T == 4)
        st.market_discarded += rem;
      else if (S == 1)
        insert_r<1>(B, st, P, rem, oid, tid, ts, tns);
      else
        insert_r<0>(B, st, P, rem, oid, tid, ts, tns);
    }
  } else {
    if (S == 1)
      cancel_r<1>(B, st, oid, Q, P);
    else
      cancel_r<0>(B, st, oid, Q, P);
  }
}

// Messages of the book: source 1 msgs[beg1, beg1 + n1), then source 2 (the step
// form's agent orders) msgs2[beg2, beg2 + n2), read in 64-message chunks (one
// record per lane) and broadcast one at a time.  l2_each: a snapshot after every
// source-1 message, into row beg1 + k.
template <bool SPILL>
__device__ __forceinline__ void process_all_r(Book<SPILL> &B, State &st, const ProcArgs &a, long long beg1,
                                              long long n1, long long beg2, long long n2, bool l2_each,
                                              int *scratch) {
  const int l = lane_id_local();
  const long long total = n1 + n2;
#pragma nounroll
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
#pragma nounroll
    for (int j = 0; j < cnt; ++j) {
      const int T = rdlane(u.x, j), S = rdlane(u.y, j), P = rdlane(u.z, j), Q = rdlane(u.w, j);
      const int oid = rdlane(v.x, j), tid = rdlane(v.y, j), ts = rdlane(v.z, j), tns = rdlane(v.w, j);
      process_msg_r(B, st, T, S, P, Q, oid, tid, ts, tns);
      if (l2_each && k0 + j < n1) write_l2_r(B, st, a.levels, a.l2_out + (beg1 + k0 + j) * 4 * a.levels, scratch);
    }
  }
}

template <bool SPILL>
__device__ __forceinline__ void run_book_r(const ProcArgs &a, int i, int2 *lds, int *scratch) {
  const int l = lane_id_local();
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
  const int row = a.out_rows ? uni(a.out_rows[i]) : i;
  st.fills = a.fills ? a.fills + (int64_t)row * a.fill_cap * kTradeFields : nullptr;
  st.fill_cap = a.fill_cap;
  st.fill_count = 0;
  st.agent_tid = a.agent_tid;

  Book<SPILL> B;
  B.lds = lds;
  B.hbm = a.books + uni64(h->book_off);
  B.W = a.W;
  B.cap = st.cap;
  // HBM -> registers (slots < RS) and LDS window (slots [RS, W))
#pragma unroll
  for (int sd = 0; sd < 2; ++sd) {
    const int n = st.n[sd];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const int s = c * kWave + l;
      Chunk x = zero_chunk();
      if (s < n) {
        x.pq = B.hbm[(int64_t)(sd * 3 + 0) * st.cap + s];
        x.ot = B.hbm[(int64_t)(sd * 3 + 1) * st.cap + s];
        x.tt = B.hbm[(int64_t)(sd * 3 + 2) * st.cap + s];
      }
      B.r[sd][c] = x;
    }
    const int nw = n < a.W ? n : a.W;
    for (int p = 0; p < 3; ++p)
      for (int base = RS; base < nw; base += kWave)
        if (base + l < nw) *B.tail(sd, p, base + l) = B.hbm[(int64_t)(sd * 3 + p) * st.cap + base + l];
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
  process_all_r(B, st, a, beg1, n1, (long long)i * a.w2, n2, a.l2_mode == 1, scratch);
  if (a.l2_mode == 2) write_l2_r(B, st, a.levels, a.l2_out + (int64_t)row * 4 * a.levels, scratch);

  // registers and LDS window -> HBM
#pragma unroll
  for (int sd = 0; sd < 2; ++sd) {
    const int n = st.n[sd];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const int s = c * kWave + l;
      if (s < n) {
        B.hbm[(int64_t)(sd * 3 + 0) * st.cap + s] = B.r[sd][c].pq;
        B.hbm[(int64_t)(sd * 3 + 1) * st.cap + s] = B.r[sd][c].ot;
        B.hbm[(int64_t)(sd * 3 + 2) * st.cap + s] = B.r[sd][c].tt;
      }
    }
    const int nw = n < a.W ? n : a.W;
    for (int p = 0; p < 3; ++p)
      for (int base = RS; base < nw; base += kWave)
        if (base + l < nw) B.hbm[(int64_t)(sd * 3 + p) * st.cap + base + l] = *B.tail(sd, p, base + l);
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
__global__ void __launch_bounds__(1024) k_process_reg(ProcArgs a) {
  extern __shared__ int2 smem[];
  const int w = uni(threadIdx.x / kWave);  // uniform: one wave = one book
  const int i = blockIdx.x * a.bpb + w;
  if (i >= a.n) return;
  int2 *lds = smem + (int64_t)w * a.lds_int2_per_wave;
  int *scratch = reinterpret_cast<int *>(lds + 6 * (a.W - RS));
  run_book_r<SPILL>(a, i, lds, scratch);
}

__global__ void k_selftest_shift(int32_t *out) {
  const int l = lane_id_local();
  const int x = 3 * l + 1;
  out[l] = shr1(x, -5);        // lane l-1; lane 0 gets the fill
  out[64 + l] = shl1(x, -7);   // lane l+1; lane 63 gets the fill
  out[128 + l] = from_lane(x, (l + 5) & 63);
}

}  // namespace

int regbook_slots() { return RS; }

hipError_t launch_process_reg(const ProcArgs &a, bool spill, hipStream_t s) {
  const int threads = a.bpb * kWave;
  const size_t lds = (size_t)a.bpb * a.lds_int2_per_wave * sizeof(int2);
  const int grid = (a.n + a.bpb - 1) / a.bpb;
  if (spill)
    hipLaunchKernelGGL(k_process_reg<true>, dim3(grid), dim3(threads), lds, s, a);
  else
    hipLaunchKernelGGL(k_process_reg<false>, dim3(grid), dim3(threads), lds, s, a);
  return hipGetLastError();
}

hipError_t set_process_reg_lds_limit(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void *)k_process_reg<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)k_process_reg<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

hipError_t launch_selftest_shift(int32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_selftest_shift, dim3(1), dim3(64), 0, s, out);
  return hipGetLastError();
}

}  // namespace lob
