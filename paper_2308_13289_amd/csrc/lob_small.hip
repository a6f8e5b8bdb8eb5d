// lob_small.hip -- matching kernel for books of capacity <= 128 orders per side.
//
// Same algorithm and results as lob_kernels.hip (one wavefront per book, each side
// kept in price-time priority, slot 0 = best), different residency: while the
// book's messages run, the whole book lives in VGPRs.  Side s is two 64-lane
// chunks (slot 64c + lane in chunk c) of four registers each: P, Q, OID of
// Section 4 and a handle H to the order's other fields (TID, Ts, Tns), which only
// the stored book needs -- the index of the message that added the order in this
// launch, or the order's slot in the book as loaded.  The book is read from one
// of its two buffers and written to the other, so the loaded copy stays readable
// until the end.  The best order is lane 0 of chunk 0;
// changing one order is a lane-select; moving orders by one slot is a DPP wave
// shift (wave_shr:1 / wave_shl:1) with the neighbouring chunk's edge lane carried
// in, and chunk 1 is left alone while the side holds at most 64 orders; removing
// several leading orders at once is a ds_bpermute.  Trade records are staged one
// per lane (lane k holds the k-th pending record) and stored to the log when 64
// are pending and at the end of every 64-message chunk, so a message that trades
// once costs four lane-selects and no store.
//
// Per 64 messages the lanes decode the message cases, check that times do not
// decrease and add the submitted limit / market quantities and the quantities
// cancels ask to remove to per-lane sums; the scalar path per message only
// dispatches on the case.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include "lob_device.h"
#include "lob_internal.h"

// v_writelane_b32 through its LLVM intrinsic (clang has no builtin for it here), so
// the compiler still sees the instruction and inserts its wait states.
__device__ int lob_writelane_i32(int value, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

namespace lob {
namespace {

using namespace dev;

constexpr int kSlots = 2 * kWave;  // orders per side the kernel holds

// Branch-layout hints: the expected outcome becomes the fall-through path.
#define LOB_LIKELY(x) __builtin_expect(!!(x), 1)
#define LOB_UNLIKELY(x) __builtin_expect(!!(x), 0)

// Lane masks of one signed compare each (a < b, a <= b, a >= b, a == b): a single
// v_cmp whose result is the mask, which the compiler cannot turn into a 0/1
// value carried across a branch and compared again.
__device__ __forceinline__ uint64_t lt_mask(int a, int b) { return __builtin_amdgcn_sicmp(a, b, 40); }
__device__ __forceinline__ uint64_t le_mask(int a, int b) { return __builtin_amdgcn_sicmp(a, b, 41); }
__device__ __forceinline__ uint64_t ge_mask(int a, int b) { return __builtin_amdgcn_sicmp(a, b, 39); }
__device__ __forceinline__ uint64_t eq_mask(int a, int b) { return __builtin_amdgcn_sicmp(a, b, 32); }

// Wait for the wave's outstanding LDS operations (lgkmcnt 0; vmcnt, expcnt left at
// their maxima), so that results of a ds_bpermute are in place before the next
// message instead of being waited for at every later use.
__device__ __forceinline__ void lds_wait() { __builtin_amdgcn_s_waitcnt(0xc07f); }

// x with lane `lane` (uniform) replaced by the uniform value v
__device__ __forceinline__ int wl(int x, int v, int lane) { return lob_writelane_i32(v, lane, x); }
// lane l receives lane l-1 (up1) or l+1 (dn1); the lane without a source receives 0
__device__ __forceinline__ int up1(int x) { return __builtin_amdgcn_mov_dpp(x, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int dn1(int x) { return __builtin_amdgcn_mov_dpp(x, 0x130, 0xf, 0xf, true); }

// One chunk: the fields of slots 64c + lane.  h: 2 * k for the order added by
// message k of this launch's stream, 2 * (-1 - s) for the order loaded from slot s;
// bit 0 set when the order carries the agent's trader id (step form).
struct Chunk {
  int p, q, o, h;
};

struct Side {
  Chunk c0, c1;
};

// TAIL form: the orders of a side past its first 128 live in LDS, worst first --
// entry t of a side holding n orders is slot n - 1 - t -- so orders enter and leave
// the register window at the tail's end, the only place top-of-book traffic touches.
struct Tail {
  int4 *a;  // (P, Q, OID, H)
};

struct Book {
  Side ask, bid;  // side 0 = asks, side 1 = bids
  Tail tl[2];     // TAIL form only
};

template <int SD>
__device__ __forceinline__ Side &side(Book &b) {
  if constexpr (SD == 0)
    return b.ask;
  else
    return b.bid;
}

__device__ __forceinline__ Chunk tail_get(const Tail &t, int i) {
  const int4 a = t.a[i];
  Chunk v;
  v.p = a.x;
  v.q = a.y;
  v.o = a.z;
  v.h = a.w;
  return v;
}

__device__ __forceinline__ void tail_put(const Tail &t, int i, const Chunk &v) {
  t.a[i] = make_int4(v.p, v.q, v.o, v.h);
}

// Tail entries [lo, hi) move by d = +1 (up) or -1 (down).  Up to four 64-entry
// groups are read before any is written, groups taken from the top for a move up
// and from the bottom for a move down, so every entry is read before the write
// that lands on it.
__device__ __forceinline__ void tail_move(const Tail &t, int lo, int hi, int d) {
  constexpr int G = 4;
  const int l = lane_id();
  if (hi <= lo) return;
  const int span = G * kWave;
  for (int k = 0; k < hi - lo; k += span) {
    // this round's entries: [r0, r0 + span) clipped to [lo, hi)
    const int r0 = d > 0 ? (hi - k - span) : (lo + k);
    Chunk v[G];
    bool mv[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int e = r0 + g * kWave + l;
      mv[g] = (e >= lo) & (e < hi);
      if (mv[g]) v[g] = tail_get(t, e);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int e = r0 + g * kWave + l;
      if (mv[g]) tail_put(t, e + d, v[g]);
    }
  }
}

// Lanes l >= k (0 <= k < 64).  TAIL form: taken straight from a scalar mask (one
// scalar shift instead of a vector compare), which measured faster there.
template <bool TAIL>
__device__ __forceinline__ bool from_k(int k) {
  if constexpr (TAIL)
    return __builtin_amdgcn_inverse_ballot_w64(~0ull << k);
  else
    return lane_id() >= k;
}

__device__ __forceinline__ void pick(Chunk &x, bool c, const Chunk &v) {
  x.p = c ? v.p : x.p;
  x.q = c ? v.q : x.q;
  x.o = c ? v.o : x.o;
  x.h = c ? v.h : x.h;
}

// Wave-uniform state of the book being processed.  The counters are this call's
// increments, added to the header's at the end; counts of trades, log records and
// missed cancels fit 32 bits because a call gives a book fewer than 2^30 messages.
struct RState {
  int n[2];
  int cap, flags;
  int small_lim;  // min(capacity, 64): below it an insert without a tail needs no other test
  int trades, misses;
  // cancel_short: of the cancelled quantities requested, the part no order gave up
  // (the request beyond the order's quantity, or all of it when no order has the id)
  long long cancel_short, market_discarded, rejected_qty;
  int last_ts, last_tns, seen;
  int32_t *log;  // the book's next free log record, or nullptr
  int log_room;  // records that still fit in the log
  int logged;    // records stored by this call
  int32_t *fills;
  int fill_cap, fill_count, agent_tid;
  uint64_t agm;  // agent fills (kAgentMask): the chunk's messages that carry the agent's trader id
};

// Agent fills: whether message j of the chunk v = (OID, TID, Ts, Tns) carries the
// agent's trader id -- a bit of the chunk's mask, or a lane read in the forms that
// are short of scalar registers (a tail, per-message L2).
template <bool TAIL, int X>
constexpr bool kAgentMask = !TAIL && (X & 2) == 0;

// Books whose times go backwards (Section 4.1: among equal prices the earlier time
// has priority, which then differs from arrival order).  Without a tail, and without
// per-message L2 or with the level-1 rows of the execution step, the kernel carries
// a second copy of its message loop whose insert compares times (kTimedInline); the
// other forms leave such a book uncommitted and mark it for the LDS engine, launched
// after them (k_process_deferred, small_defers), which keeps each order's time
// beside it.  Either way the hot loop holds no code for it.
template <bool TAIL, int X>
constexpr bool kTimedInline = !TAIL && ((X & 2) == 0 || (X & 16) != 0);

// The next message's case read one message ahead, off the dispatch's dependency
// chain, for two more scalar moves per message: faster where few waves share a SIMD
// (the TAIL form's large books, the rotating variant's 2 to 4 waves per SIMD) and
// latency bounds a book; slower with agent fills, and with 8 or more waves per SIMD
// (the variant without rotation), where issue does.
template <bool TAIL, int X>
constexpr bool kReadAhead = (X & 1) == 0 && (TAIL || (X & 4) != 0);

// The chunk-0 insert of a side of fewer than 64 orders as its own path: always
// without a tail; with one only in the instantiation for books that the flow drains
// (X bit 3): it saves the tail form's work on chunk 1 there, and costs books that
// stay deep 6-9% (register copies where the paths merge), so the autotuner picks
// the instantiation per batch.
template <bool TAIL, int X>
constexpr bool kChunk0Insert = !TAIL || (X & 8) != 0;

template <bool TAIL, int X>
__device__ __forceinline__ bool agent_msg(const RState &st, const int4 &v, int j) {
  if constexpr (kAgentMask<TAIL, X>)
    return ((st.agm >> j) & 1) != 0;
  else
    return rdlane(v.y, j) == st.agent_tid;
}

// Pending trade records, one per lane; k of them (uniform) are pending.  A record
// keeps the standing order's price, the fill and the standing id; the aggressor's
// id and time are those of message j of the current chunk, fetched when the
// records are stored, which happens at the latest when the chunk ends.  When the
// launch collects agent fills, bit 6 of j is set for a standing order of the agent.
struct Stage {
  int p, q, po, j;
  int k;
  // per-lane running sums of submitted limit and market quantities, of the
  // quantities cancel messages ask to remove and of traded quantities, reduced over
  // the wave once at the end of the call
  unsigned long long limit_qty, market_qty, traded_qty, cancel_qty;
};

// Sum over the wave of a non-negative int32 per lane, as 64-bit.
__device__ __forceinline__ long long wave_sum(int v) {
  const int lo = scan_incl(v & 0xffff);
  const int hi = scan_incl((int)((unsigned)v >> 16));
  return (long long)rdlane(lo, 63) + ((long long)rdlane(hi, 63) << 16);
}

// Sum over the wave of a 64-bit value per lane (the total below 2^63).
__device__ __forceinline__ long long wave_sum64(unsigned long long v) {
  return wave_sum((int)(unsigned)v) + (wave_sum((int)(unsigned)(v >> 32)) << 32);
}

// The pending trades are counted (trades and traded quantity) and stored; v holds
// (OID, TID, Ts, Tns) of the chunk's messages across the lanes.  X bit 0: the
// trades in which the agent takes part (a standing order of the agent, or an
// aggressor carrying its trader id) are also stored as agent fills, in order.
template <bool TAIL, int X>
__device__ __forceinline__ void flush(RState &st, Stage &sg, const int4 &v) {
  if (sg.k == 0) return;
  st.trades += sg.k;
  const int l = lane_id();
  sg.traded_qty += (unsigned)(l < sg.k ? sg.q : 0);
  const int jj = (X & 1) != 0 ? (sg.j & 63) : sg.j;
  if (st.log) {
    const int stored = st.log_room < sg.k ? st.log_room : sg.k;
    const int ao = from_lane(v.x, jj), ts = from_lane(v.z, jj), tns = from_lane(v.w, jj);
    if (l < stored) {
      int2 *r = reinterpret_cast<int2 *>(st.log + l * kTradeFields);
      r[0] = make_int2(sg.p, sg.q);
      r[1] = make_int2(sg.po, ao);
      r[2] = make_int2(ts, tns);
    }
    if (stored < sg.k) st.flags |= kFlagTradeFull;
    st.log += stored * kTradeFields;
    st.log_room -= stored;
    st.logged += stored;
    lds_wait();  // the permutes are complete on every path out
  }
  if constexpr ((X & 1) != 0) {
    if (st.fills) {
      bool agg;  // the aggressor carries the agent's trader id
      if constexpr (kAgentMask<TAIL, X>) {
        agg = ((st.agm >> jj) & 1) != 0;
      } else {
        agg = from_lane(v.y, jj) == st.agent_tid;
        lds_wait();
      }
      const bool ag = (l < sg.k) & (agg | ((sg.j & 64) != 0));
      const uint64_t ma = ballot(ag);
      if (ma) {
        const int ao = from_lane(v.x, jj), ts = from_lane(v.z, jj), tns = from_lane(v.w, jj);
        const int f = st.fill_count + popc(ma & mask_lt());
        if (ag && f < st.fill_cap) {
          int2 *r = reinterpret_cast<int2 *>(st.fills + (int64_t)f * kTradeFields);
          r[0] = make_int2(sg.p, sg.q);
          r[1] = make_int2(sg.po, ao);
          r[2] = make_int2(ts, tns);
        }
        st.fill_count += popc(ma);
        lds_wait();
      }
    }
  }
  sg.k = 0;
}

// One trade from uniform values; the aggressor is message j of the chunk v (with
// bit 6 set for a standing order of the agent when the launch collects fills).
template <bool TAIL, int X>
__device__ __forceinline__ void stage_one(RState &st, Stage &sg, int P, int fill, int po, int j, const int4 &v) {
  sg.p = wl(sg.p, P, sg.k);
  sg.q = wl(sg.q, fill, sg.k);
  sg.po = wl(sg.po, po, sg.k);
  sg.j = wl(sg.j, j, sg.k);
  if (LOB_UNLIKELY(++sg.k == kWave)) flush<TAIL, X>(st, sg, v);
}

// ntr trades held by lanes [0, ntr) (P, fill, standing id per lane; the aggressor
// is message j of the chunk v): rotate them behind the pending ones.  pa: per lane,
// the standing order is the agent's (used when the launch collects fills).
template <bool TAIL, int X>
__device__ __forceinline__ void stage_many(RState &st, Stage &sg, int ntr, int P, int fill, int po, int j, bool pa,
                                           const int4 &v) {
  const int l = lane_id();
  const int src = (l - sg.k) & 63;
  const int rp = from_lane(P, src), rq = from_lane(fill, src), ro = from_lane(po, src);
  int rj = j;
  if constexpr ((X & 1) != 0) rj = from_lane(j | (pa ? 64 : 0), src);
  const bool mine = l >= sg.k;
  sg.p = mine ? rp : sg.p;
  sg.q = mine ? rq : sg.q;
  sg.po = mine ? ro : sg.po;
  sg.j = mine ? rj : sg.j;
  const int end = sg.k + ntr;
  if (end >= kWave) {
    sg.k = kWave;
    flush<TAIL, X>(st, sg, v);
    sg.p = rp;
    sg.q = rq;
    sg.po = ro;
    sg.j = rj;
    sg.k = end - kWave;
  } else {
    sg.k = end;
  }
}

__device__ __forceinline__ Chunk edge(const Chunk &x, int lane) {  // uniform fields of one lane
  Chunk v;
  v.p = rdlane(x.p, lane);
  v.q = rdlane(x.q, lane);
  v.o = rdlane(x.o, lane);
  v.h = rdlane(x.h, lane);
  return v;
}

// Lanes with `take` receive the next lane's order (dn) or the previous lane's (up).
// MASKED: one DPP move per field, in place, with only those lanes active (no
// select).  A lane whose source lane is inactive or outside the wave then gets no
// defined value, so the callers' masks make every such lane one that is overwritten
// or unused: shift_dn takes lanes l >= k (each source, lane l + 1, is active, except
// that lane 63's is outside the wave), shift_up takes lanes l >= at and the new
// order is then written into lane at.  Otherwise every lane moves and a select
// keeps the lanes without `take`.  The register-only form uses MASKED (4 VALU fewer
// per shift); the TAIL form measured faster with the select.
template <bool MASKED>
__device__ __forceinline__ void shift_dn(Chunk &x, bool take) {
  if constexpr (MASKED) {
    if (take) {
      x.p = dn1(x.p);
      x.q = dn1(x.q);
      x.o = dn1(x.o);
      x.h = dn1(x.h);
    }
  } else {
    const int p = dn1(x.p), q = dn1(x.q), o = dn1(x.o), h = dn1(x.h);
    x.p = take ? p : x.p;
    x.q = take ? q : x.q;
    x.o = take ? o : x.o;
    x.h = take ? h : x.h;
  }
}

// Every lane takes the next lane's order (lane 63 receives zeros).
__device__ __forceinline__ void shift_dn_all(Chunk &x) {
  x.p = dn1(x.p);
  x.q = dn1(x.q);
  x.o = dn1(x.o);
  x.h = dn1(x.h);
}

template <bool MASKED>
__device__ __forceinline__ void shift_up(Chunk &x, bool take) {
  if constexpr (MASKED) {
    if (take) {
      x.p = up1(x.p);
      x.q = up1(x.q);
      x.o = up1(x.o);
      x.h = up1(x.h);
    }
  } else {
    const int p = up1(x.p), q = up1(x.q), o = up1(x.o), h = up1(x.h);
    x.p = take ? p : x.p;
    x.q = take ? q : x.q;
    x.o = take ? o : x.o;
    x.h = take ? h : x.h;
  }
}

// lane `lane` of x takes the uniform order v
__device__ __forceinline__ void put(Chunk &x, const Chunk &v, int lane) {
  x.p = wl(x.p, v.p, lane);
  x.q = wl(x.q, v.q, lane);
  x.o = wl(x.o, v.o, lane);
  x.h = wl(x.h, v.h, lane);
}

// Slots (k, n) of a side move down by one (slot k < 128 is dropped); in the TAIL
// form the tail's last entry (slot 128) moves up into slot 127.
// FRONT: k is 0 (the best order), every lane moves without a select (used in the
// TAIL form; without a tail the select form measured faster).
template <bool TAIL, bool FRONT = false>
__device__ __forceinline__ void remove_at(Side &S, const Tail &tl, int k, int n) {
  const int l = lane_id();
  constexpr bool front = FRONT;
  if (TAIL ? LOB_LIKELY(n > kWave) : LOB_UNLIKELY(n > kWave)) {
    const Chunk in = edge(S.c1, 0);  // slot 64 moves to slot 63
    if (front) {
      shift_dn_all(S.c1);
      shift_dn_all(S.c0);
      put(S.c0, in, 63);
    } else {
      shift_dn<!TAIL>(S.c1, l + kWave >= k);
      if (k < kWave) {
        shift_dn<!TAIL>(S.c0, from_k<TAIL>(k));
        put(S.c0, in, 63);
      }
    }
    if constexpr (TAIL) {
      if (n > kSlots) pick(S.c1, l == 63, tail_get(tl, n - kSlots - 1));
    }
  } else if (front) {
    shift_dn_all(S.c0);
  } else {
    shift_dn<!TAIL>(S.c0, from_k<TAIL>(k));
  }
}

__device__ __forceinline__ void shift_front(Side &S, int m, int n);

// The first m slots of a side (1 <= m <= 128) are removed: slot s takes slot s + m;
// in the TAIL form the register positions freed at the end take the tail's last
// entries.
template <bool TAIL>
__device__ __forceinline__ void remove_front(Side &S, const Tail &tl, int m, int n) {
  if (m == 1) {
    remove_at<TAIL, TAIL>(S, tl, 0, n);
    return;
  }
  const int l = lane_id();
  const int nr = n < kSlots ? n : kSlots;
  if (m < nr) shift_front(S, m, nr);
  if constexpr (TAIL) {
    if (n > kSlots) {
      const int T = n - kSlots, k = m < T ? m : T, base = kSlots - m;
      const int j0 = l - base, j1 = kWave + l - base;  // tail index T-1-j lands in position base + j
      const bool t0 = (j0 >= 0) & (j0 < k), t1 = (j1 >= 0) & (j1 < k);
      pick(S.c0, t0, tail_get(tl, t0 ? T - 1 - j0 : T - 1));
      pick(S.c1, t1, tail_get(tl, t1 ? T - 1 - j1 : T - 1));
    }
  }
}

// Register slots [m, nr) move to [0, nr - m) (2 <= m < nr <= 128).
__device__ __forceinline__ void shift_front(Side &S, int m, int n) {
  const int l = lane_id();
  const int src = (l + m) & 63;
  if (n <= kWave) {
    S.c0.p = from_lane(S.c0.p, src);
    S.c0.q = from_lane(S.c0.q, src);
    S.c0.o = from_lane(S.c0.o, src);
    S.c0.h = from_lane(S.c0.h, src);
    lds_wait();
    return;
  }
  Chunk a, b;
  a.p = from_lane(S.c0.p, src);
  a.q = from_lane(S.c0.q, src);
  a.o = from_lane(S.c0.o, src);
  a.h = from_lane(S.c0.h, src);
  b.p = from_lane(S.c1.p, src);
  b.q = from_lane(S.c1.q, src);
  b.o = from_lane(S.c1.o, src);
  b.h = from_lane(S.c1.h, src);
  if (m < kWave) {
    const bool low = l + m < kWave;  // the source slot is in the same chunk
    S.c0.p = low ? a.p : b.p;
    S.c0.q = low ? a.q : b.q;
    S.c0.o = low ? a.o : b.o;
    S.c0.h = low ? a.h : b.h;
    S.c1 = b;
  } else {
    S.c0 = b;  // slot l takes slot 64 + (l + m - 64)
  }
  lds_wait();
}

// Matching loop of Section 4.1 against side OPP (0 asks, 1 bids) for an aggressor
// with limit price lim and quantity q.  Returns the unfilled quantity.
// X: what the launch collects besides trades and final L2 -- bit 0 agent fills,
// bit 1 per-message L2 (the checks for what it does not collect are compiled out);
// bit 2 selects the rotating-priority variant, bit 3 the TAIL form's chunk-0 insert.
// LIMIT: a limit order that crosses (the caller has tested rests_apart).
// The aggressor is message j of the chunk v = (OID, TID, Ts, Tns) across the lanes.
template <int OPP, bool TAIL, int X, bool LIMIT>
__device__ __forceinline__ int match(Book &bk, RState &st, Stage &sg, int lim, int q, const int4 &v, int j) {
  Side &S = side<OPP>(bk);
  const Tail &tl = bk.tl[OPP];
  int n = st.n[OPP];
  constexpr bool buyer = (OPP == 0);
  // a limit order gets here only when it crosses (rests_apart is false)
  if constexpr (!LIMIT) {
    if (LOB_UNLIKELY(n == 0)) return q;  // q > 0: the decode turns messages with Q <= 0 into no-ops
    const int bp0 = rdlane(S.c0.p, 0);
    if (LOB_UNLIKELY(buyer ? bp0 > lim : bp0 < lim)) return q;
  }
  const int bp = rdlane(S.c0.p, 0);
  const int bq = rdlane(S.c0.q, 0);
  if (LOB_LIKELY(q <= bq)) {
    // Q_s' = Q_s - Q_a >= 0: one trade with the best order fills the aggressor
    const int bo = rdlane(S.c0.o, 0);
    stage_one<TAIL, X>(st, sg, bp, q, bo, (X & 1) != 0 ? j | ((rdlane(S.c0.h, 0) & 1) << 6) : j, v);
    if (q < bq) {
      S.c0.q = wl(S.c0.q, bq - q, 0);
    } else {
      remove_at<TAIL, TAIL>(S, tl, 0, n);
      st.n[OPP] = n - 1;
    }
    return 0;
  }
  // the aggressor outlasts the best order: one prefix scan per chunk of crossing
  // orders; in the TAIL form a register window consumed whole is refilled from the
  // tail and the scan goes on
  const int l = lane_id();
  for (;;) {
    const int nr = n < kSlots ? n : kSlots;
    int removed = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (c == 1 && (removed < kWave || nr <= kWave || q == 0)) break;
      Chunk &F = c == 0 ? S.c0 : S.c1;
      const bool valid = c * kWave + l < nr;
      const bool at = buyer ? F.p <= lim : F.p >= lim;
      const uint64_t mc = ballot(valid) & ballot(at);
      const bool cross = valid & at;
      const int qv = cross ? F.q : 0;
      // running sums of the crossing quantities; excl is exact wherever it is below q
      int incl, excl;
      if (LOB_LIKELY(q < kScanExactQ)) {
        const int qc = min(qv, q + 1);
        incl = scan_incl(qc);
        excl = incl - qc;
      } else {
        incl = scan_incl_sat(qv);
        excl = shr1(incl, 0);
      }
      const bool takes = cross & (excl < q);
      const uint64_t mt = mc & ballot(excl < q);
      if (mt == 0) break;
      const int ntr = popc(mt);
      const int room = q - excl;
      const bool full = takes & (qv <= room);
      const int nfull = popc(ballot(full));
      const int fill = takes ? min(qv, room) : 0;
      stage_many<TAIL, X>(st, sg, ntr, F.p, fill, F.o, j, (F.h & 1) != 0, v);
      F.q = (takes & !full) ? F.q - fill : F.q;  // the partially filled order, if any
      const int consumed = (nfull == ntr) ? rdlane(incl, ntr - 1) : q;
      q -= consumed;
      removed += nfull;
      if (nfull < kWave) break;
    }
    if (removed > 0) {
      remove_front<TAIL>(S, tl, removed, n);
      n -= removed;
      st.n[OPP] = n;
    }
    if (!TAIL || removed < kSlots || q == 0 || n == 0) break;
  }
  return q;
}

// Where the stream of the book being processed lives (for the handles' records).
struct Streams {
  const int32_t *msgs, *msgs2;
  long long beg1, n1, beg2, total;
};

// Where every order's time is kept: the records of this launch's stream for orders
// it added, the loaded book (the buffer this launch does not write) for the others.
struct Origin {
  Streams m;
  const int2 *hb;  // the loaded book, both sides
  int cap;
};

// The message loop carries the addresses of those times packed into the lanes of
// one VGPR (lane k holds 32-bit word k), read back with ds_bpermute into VGPRs only on
// the rare path that needs them: held in scalar registers they would raise the
// kernel's register count, and its occupancy, for a path that almost never runs.
// Words 0-1: record 0 of source 1; 2-3: where record k of source 2 sits for k >= n1;
// 4: n1; 5-6 and 7-8: the (Ts, Tns) arrays of the loaded ask and bid sides.
__device__ __forceinline__ int pack_origin(const Origin &g) {
  const uint64_t b1 = (uint64_t)(uintptr_t)g.m.msgs + (uint64_t)g.m.beg1 * (kMsgFields * 4);
  const uint64_t b2 = (uint64_t)(uintptr_t)g.m.msgs2 + (uint64_t)(g.m.beg2 - g.m.n1) * (kMsgFields * 4);
  const uint64_t t0 = (uint64_t)(uintptr_t)(g.hb + 2 * (int64_t)g.cap);
  const uint64_t t1 = (uint64_t)(uintptr_t)(g.hb + 5 * (int64_t)g.cap);
  const uint32_t w[9] = {(uint32_t)b1, (uint32_t)(b1 >> 32), (uint32_t)b2, (uint32_t)(b2 >> 32), (uint32_t)g.m.n1,
                         (uint32_t)t0, (uint32_t)(t0 >> 32), (uint32_t)t1, (uint32_t)(t1 >> 32)};
  int pk = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) pk = wl(pk, (int)w[k], k);
  asm volatile("" : "+v"(pk));  // opaque: the words are read back from the lanes
  return pk;
}

// Address of the (Ts, Tns) of the order with handle h on side sd, one per lane.  Must
// run with every lane of the wave active: a ds_bpermute reads zero from an inactive
// source lane.  h may be anything; the address is valid only where an order is held.
__device__ __forceinline__ const int2 *time_addr(int h, int pk, int sd) {
  const int idx = h >> 1;
  const int n1 = from_lane(pk, 4);
  const int w = idx >= 0 ? (idx < n1 ? 0 : 2) : 5 + 2 * sd;
  const uint64_t base = (uint64_t)(uint32_t)from_lane(pk, w) | (uint64_t)(uint32_t)from_lane(pk, w + 1) << 32;
  const uint64_t off = idx >= 0 ? (uint64_t)idx * (kMsgFields * 4) + 24 : (uint64_t)(-1 - idx) * 8;
  return reinterpret_cast<const int2 *>(base + off);
}

// Whether each held order (p, handle h; held: this lane holds an order) is ahead of
// a new order (P, ts, tns) on side SD under price-time priority: a better price, or
// the same price and a time at or before (ts, tns) (equal times: the standing order
// arrived first).  For books whose times went backwards; otherwise every standing
// order is at most as old as the new one and an equal price alone puts it ahead.
// Every lane of the wave active (time_addr).
template <int SD>
__device__ __forceinline__ bool ahead_timed(bool held, int p, int h, int P, int ts, int tns, int pk) {
  const int2 *ta = time_addr(h, pk, SD);
  bool ahead = held & (SD == 1 ? p > P : p < P);
  if (held & (p == P)) {
    const int2 t = *ta;
    ahead = (t.x < ts) | ((t.x == ts) & (t.y <= tns));
  }
  return ahead;
}

// Whether a limit order at price lim meets no standing order of side OPP: the side
// is empty or its best price does not overlap lim.  Lane 0 is read before the count
// is tested (it holds some value either way), so that the common outcome, a best
// price apart from lim, takes one test.
template <int OPP>
__device__ __forceinline__ bool rests_apart(const Book &bk, const RState &st, int lim) {
  const Side &S = OPP == 0 ? bk.ask : bk.bid;
  const int bp = rdlane(S.c0.p, 0);
  if (LOB_LIKELY(OPP == 0 ? bp > lim : bp < lim)) return true;
  return st.n[OPP] == 0;
}

// Add (Section 4.1, item 1) on side SD: the new order goes to its price-time
// position.  While a book's times have never gone backwards every standing order is
// at most as old as the new one, so that position is behind every order with an
// equal or better price; in a book flagged for times going backwards (TIMED) the
// times of the orders at the new order's price are compared too (ahead_timed).
// hnd: the new order's handle; it is message j of the chunk v = (OID, TID, Ts, Tns).
template <int SD, bool TAIL, bool TIMED, bool CHUNK0 = !TAIL>
__device__ __forceinline__ void insert(Book &bk, RState &st, int P, int Q, int oid, int hnd, const int4 &v_,
                                       int j, int pk) {
  static_assert(!(TAIL && TIMED), "the TAIL form leaves such books to the LDS engine");
  Side &S = side<SD>(bk);
  const Tail &tl = bk.tl[SD];
  const int l = lane_id();
  const int n = st.n[SD];
  if constexpr (CHUNK0 && !TIMED) {
    // a side of fewer than 64 orders (without a tail the rule; with one, a book the
    // flow has drained): only chunk 0 takes part, and one test covers the capacity
    if (LOB_LIKELY(n < st.small_lim)) {
      const uint64_t live = (1ull << n) - 1;  // n < 64 here
      const int at = popc(live & (SD == 1 ? ge_mask(S.c0.p, P) : le_mask(S.c0.p, P)));
      Chunk v;
      v.p = P;
      v.q = Q;
      v.o = oid;
      v.h = hnd;
      shift_up<!TAIL>(S.c0, l >= at);
      put(S.c0, v, at);
      st.n[SD] = n + 1;
      return;
    }
  }
  if (LOB_UNLIKELY(n >= st.cap)) {
    st.rejected_qty += (unsigned)Q;
    st.flags |= kFlagSideFull;
    return;
  }
  const int nr = n < kSlots ? n : kSlots;
  // the orders ahead form a prefix, so chunk 1 holds some only when chunk 0 is all
  // ahead: both counts add up without a test (without a tail chunk 1 is rarely in
  // use and is skipped while it is empty)
  int ts = 0, tns = 0;
  int pos;
  if constexpr (TIMED) {
    ts = rdlane(v_.z, j);
    tns = rdlane(v_.w, j);
    pos = popc(ballot(ahead_timed<SD>(l < nr, S.c0.p, S.c0.h, P, ts, tns, pk)));
    if (nr > kWave) pos += popc(ballot(ahead_timed<SD>(l + kWave < nr, S.c1.p, S.c1.h, P, ts, tns, pk)));
  } else {
    pos = popc(lt_mask(l, nr) & (SD == 1 ? ge_mask(S.c0.p, P) : le_mask(S.c0.p, P)));
    if (TAIL || LOB_UNLIKELY(nr > kWave))
      pos += popc(lt_mask(l + kWave, nr) & (SD == 1 ? ge_mask(S.c1.p, P) : le_mask(S.c1.p, P)));
  }
  Chunk v;
  v.p = P;
  v.q = Q;
  v.o = oid;
  v.h = hnd;
  if constexpr (TAIL) {
    if (LOB_UNLIKELY(pos == kSlots)) {
      // behind every register order: into the tail.  The tail orders ahead of it
      // (equal or better price) are the entries [T - c, T); they move up by one and
      // the new order takes entry T - c.
      const int T = n - kSlots;
      // the orders ahead form a suffix: count from the top, 64 entries at a time,
      // until an entry is not ahead
      int c = 0;
      for (int top = T; top > 0; top -= kWave) {
        const int t = top - 1 - l;
        bool ahead = false;
        if (t >= 0) {
          const int p = tl.a[t].x;
          ahead = SD == 1 ? p >= P : p <= P;
        }
        const int k = popc(ballot(ahead));
        c += k;
        if (k < kWave) break;
      }
      tail_move(tl, T - c, T, 1);
      if (l == 0) tail_put(tl, T - c, v);
      st.n[SD] = n + 1;
      return;
    }
    // the register window is full: its last order moves to the tail's end
    if (n >= kSlots) {
      const Chunk last = edge(S.c1, 63);
      if (l == 0) tail_put(tl, n - kSlots, last);
    }
  }
  // (without a tail a side rarely holds 64 orders or more: chunk 1 work is laid out
  // of line; with one it is the common case)
  if (TAIL ? LOB_LIKELY(nr >= kWave) : LOB_UNLIKELY(nr >= kWave)) {
    // chunk 1 changes: slot 63 moves into slot 64, or the new order lands there
    const Chunk in = edge(S.c0, 63);
    shift_up<!TAIL>(S.c1, l + kWave >= pos);
    if (pos < kWave) put(S.c1, in, 0);
  }
  if (LOB_LIKELY(pos < kWave)) {
    shift_up<!TAIL>(S.c0, from_k<TAIL>(pos));
    put(S.c0, v, pos);
  } else {
    put(S.c1, v, pos - kWave);
  }
  st.n[SD] = n + 1;
}

// The best-priority tail entry with pred (the highest entry index), -1 if none.
template <typename Pred>
__device__ __forceinline__ int tail_find(int T, Pred pred) {
  const int l = lane_id();
  for (int base = (T - 1) & ~63; base >= 0; base -= kWave) {
    const int t = base + l;
    const uint64_t m = ballot((t < T) && pred(t));
    if (m) return base + 63 - __builtin_clzll(m);
  }
  return -1;
}

// Cancel / delete (Section 4.1, item 2; Section 5.1.1 for initial orders) on side SD.
// The message's price (lane j of pz, used only when no order has the id) is read on
// that rare path alone.
template <int SD, bool TAIL>
__device__ __forceinline__ void cancel(Book &bk, RState &st, int oid, int qty, int pz, int j) {
  Side &S = side<SD>(bk);
  const Tail &tl = bk.tl[SD];
  const int l = lane_id();
  const int n = st.n[SD];
  const int nr = n < kSlots ? n : kSlots;
  int k = -1;
  uint64_t m = lt_mask(l, n) & eq_mask(S.c0.o, oid);  // (l < 64: the same as l < nr)
  if (LOB_LIKELY(m != 0)) {
    // the common case, an order in chunk 0 found by its id
    const int k0 = first_set(m);
    const int Q = rdlane(S.c0.q, k0);
    if (LOB_LIKELY(Q > qty)) {
      S.c0.q = wl(S.c0.q, Q - qty, k0);
    } else {
      st.cancel_short += (unsigned)(qty - Q);
      remove_at<TAIL>(S, tl, k0, n);
      st.n[SD] = n - 1;
    }
    return;
  }
  if (nr > kWave) {
    m = lt_mask(l + kWave, nr) & eq_mask(S.c1.o, oid);
    if (m) k = kWave + first_set(m);
  }
  int t = -1;  // TAIL: entry in the tail
  if constexpr (TAIL) {
    if (k < 0 && n > kSlots) t = tail_find(n - kSlots, [&](int e) { return tl.a[e].z == oid; });
  }
  if (k < 0 && t < 0) {
    asm volatile("" : "+v"(pz));  // keeps the read below from being hoisted to the common path
    const int price = rdlane(pz, j);
    m = lt_mask(l, nr) & le_mask(S.c0.o, -9000) & eq_mask(S.c0.p, price);
    if (m) {
      k = first_set(m);
    } else if (nr > kWave) {
      m = lt_mask(l + kWave, nr) & le_mask(S.c1.o, -9000) & eq_mask(S.c1.p, price);
      if (m) k = kWave + first_set(m);
    }
    if constexpr (TAIL) {
      if (k < 0 && n > kSlots)
        t = tail_find(n - kSlots, [&](int e) { return tl.a[e].z <= -9000 && tl.a[e].x == price; });
    }
  }
  if (k < 0 && t < 0) {
    st.misses++;
    st.cancel_short += (unsigned)qty;
    return;
  }
  if constexpr (TAIL) {
    if (t >= 0) {
      const int T = n - kSlots;
      const int4 e = tl.a[t];
      const int P = uni(e.x), Q = uni(e.y);
      const int left = Q - qty;
      if (left > 0) {
        if (l == 0) tl.a[t] = make_int4(P, left, uni(e.z), uni(e.w));
      } else {
        st.cancel_short += (unsigned)(qty - Q);
        tail_move(tl, t + 1, T, -1);  // the entries above it (better priority) move down by one
        st.n[SD] = n - 1;
      }
      return;
    }
  }
  const bool lo = k < kWave;
  const int kl = k & 63;
  const int Q = lo ? rdlane(S.c0.q, kl) : rdlane(S.c1.q, kl);
  const int left = Q - qty;
  if (left > 0) {
    if (lo)
      S.c0.q = wl(S.c0.q, left, kl);
    else
      S.c1.q = wl(S.c1.q, left, kl);
  } else {
    st.cancel_short += (unsigned)(qty - Q);
    remove_at<TAIL>(S, tl, k, n);
    st.n[SD] = n - 1;
  }
}

// L2 of one side: the first L distinct prices with their summed quantities into
// out[0..L) as (price, qty); missing levels (-1, 0).  A level is a run of equal
// prices in priority order; its quantity is the exact sum of the run, capped at
// INT_MAX (level_qty).  The slots are taken 64 at a time in priority order: the two
// register chunks, then (TAIL form) the tail.
template <bool TAIL>
__device__ __forceinline__ void l2_side(const Side &S, const Tail &tl, int n, int L, int2 *out) {
  const int l = lane_id();
  const int nr = n < kSlots ? n : kSlots;
  int levels = 0;
  long long carry = 0;
  const int nchunks = TAIL ? (n + kWave - 1) / kWave : 2;
  for (int c = 0; c < nchunks && levels < L; ++c) {
    if (c * kWave >= n) break;
    const int s = c * kWave + l;
    const bool valid = s < n;
    int p, q, next;
    if (c < 2) {
      const Chunk &F = c == 0 ? S.c0 : S.c1;
      p = F.p;
      q = F.q;
      int next_in = 0;  // the price of slot 64(c+1)
      if (c == 0 && nr > kWave) next_in = rdlane(S.c1.p, 0);
      if constexpr (TAIL) {
        if (c == 1 && n > kSlots) next_in = uni(tl.a[n - kSlots - 1].x);
      }
      next = shl1(p, next_in);
    } else {
      // slot s is tail entry n - 1 - s
      p = valid ? tl.a[n - 1 - s].x : 0;
      q = valid ? tl.a[n - 1 - s].y : 0;
      next = (s + 1 < n) ? tl.a[n - 2 - s].x : 0;
    }
    const bool is_last = valid & ((s + 1 == n) | (next != p));
    const uint64_t ml = ballot(is_last);
    const int lq = level_qty(valid ? q : 0, ml, carry);
    const int lev = levels + popc(ml & mask_lt());
    if (is_last && lev < L) out[lev] = make_int2(p, lq);
    levels += popc(ml);
  }
  const int have = levels < L ? levels : L;
  if (l >= have && l < L) out[l] = make_int2(-1, 0);
}

template <bool TAIL>
__device__ __forceinline__ void write_l2(const Book &bk, const RState &st, int L, int32_t *row) {
  int2 *o = reinterpret_cast<int2 *>(row);
  l2_side<TAIL>(bk.ask, bk.tl[0], st.n[0], L, o);
  l2_side<TAIL>(bk.bid, bk.tl[1], st.n[1], L, o + L);
}

// write_l2 with L = 1 (the per-message rows of the execution environment): each
// side's best price and the exact quantity resting at it, min(sum, INT_MAX); an empty
// side has quantity 0 and an unspecified price (the execution step tells the sides
// apart by quantity).  A side is sorted by price, so the best level is every slot
// holding slot 0's price; lane l adds its two register slots (l and 64 + l) and one
// saturating scan per side sums the lanes (saturating adds of non-negative values
// give min(sum, INT_MAX) in any order), the two sides' scans independent of each
// other; when neither best price has a second order, slot 0's quantities are the
// sums and the scans are skipped.  With a tail, a level that goes on past slot 127
// takes the general form.
__device__ __forceinline__ int l1_lane_qty(const Side &S, int n, int p0) {
  const int l = lane_id();
  const int x = l < n && S.c0.p == p0 ? S.c0.q : 0;
  const int y = l + kWave < n && S.c1.p == p0 ? S.c1.q : 0;
  return sat_add(x, y);
}

template <bool TAIL>
__device__ __forceinline__ void write_l1(const Book &bk, const RState &st, int32_t *row) {
  const int l = lane_id();
  const int na = st.n[0], nb = st.n[1];
  const int pa = rdlane(bk.ask.c0.p, 0), pb = rdlane(bk.bid.c0.p, 0);
  if constexpr (TAIL) {
    if (LOB_UNLIKELY((na > kSlots && rdlane(bk.ask.c1.p, kWave - 1) == pa) ||
                     (nb > kSlots && rdlane(bk.bid.c1.p, kWave - 1) == pb))) {
      write_l2<TAIL>(bk, st, 1, row);
      return;
    }
  }
  // lane 1 of a side of one order holds a stale price: the count decides first
  const int pa1 = rdlane(bk.ask.c0.p, 1), pb1 = rdlane(bk.bid.c0.p, 1);
  const int qa0 = rdlane(bk.ask.c0.q, 0), qb0 = rdlane(bk.bid.c0.q, 0);
  int qa, qb;
  if (LOB_LIKELY((na <= 1 || pa1 != pa) && (nb <= 1 || pb1 != pb))) {
    // the common case: at most one order at each best price
    qa = na > 0 ? qa0 : 0;
    qb = nb > 0 ? qb0 : 0;
  } else {
    const int sa = scan_incl_sat(l1_lane_qty(bk.ask, na, pa));
    const int sb = scan_incl_sat(l1_lane_qty(bk.bid, nb, pb));
    qa = rdlane(sa, kWave - 1);
    qb = rdlane(sb, kWave - 1);
  }
  // the row in lanes 0-3 by lane writes: no lane-dependent selects, which the compiler
  // lays out as branches under exec masks
  int r = wl(0, pa, 0);
  r = wl(r, qa, 1);
  r = wl(r, pb, 2);
  r = wl(r, qb, 3);
  if (l < 4) row[l] = r;
}

// Handle of the order added by message k (j of the chunk v): 2k, plus 1 when the
// launch collects agent fills and the message carries the agent's trader id.
template <bool TAIL, int X>
__device__ __forceinline__ int handle(const RState &st, int k, const int4 &v, int j) {
  int h = k * 2;
  if constexpr ((X & 1) != 0) h += agent_msg<TAIL, X>(st, v, j) ? 1 : 0;
  return h;
}

// One message (Section 4.2) given its case code: 0/1 limit sell/buy, 2/3
// cancel-or-delete on the ask/bid side, 4/5 market sell/buy, 7 not processed.  Limit:
// match, then rest the remainder as one new order (item 1); market: match at
// price 0 (sell) / max_int (buy), drop the rest (item 3); cancel and delete are
// the same operation (item 2).  One straight call sequence per case, so that no
// flag derived from the case has to survive across branches.
// Message j of the chunk held as u = (type, side, P, Q), v = (oid, tid, ts, tns)
// across the lanes, message k of the book's stream; each case reads only the
// fields it uses.
template <bool TAIL, int X, bool TIMED>
__device__ __forceinline__ void process_msg(Book &bk, RState &st, Stage &sg, int code, const int4 &u, const int4 &v,
                                            int j, int k, int pk) {
  // tested in order of frequency: limit orders, cancels, market orders
  if (LOB_LIKELY(code < 2)) {
    const int P = rdlane(u.z, j), Q = rdlane(u.w, j);
    __builtin_assume(Q > 0);  // the decode gives messages with Q <= 0 code 7
    // most limit orders meet no standing order and rest whole
    if (code == 0) {
      const int rem = rests_apart<1>(bk, st, P) ? Q : match<1, TAIL, X, true>(bk, st, sg, P, Q, v, j);
      if (rem > 0)
        insert<0, TAIL, TIMED, kChunk0Insert<TAIL, X>>(bk, st, P, rem, rdlane(v.x, j), handle<TAIL, X>(st, k, v, j),
                                                       v, j, pk);
    } else {
      const int rem = rests_apart<0>(bk, st, P) ? Q : match<0, TAIL, X, true>(bk, st, sg, P, Q, v, j);
      if (rem > 0)
        insert<1, TAIL, TIMED, kChunk0Insert<TAIL, X>>(bk, st, P, rem, rdlane(v.x, j), handle<TAIL, X>(st, k, v, j),
                                                       v, j, pk);
    }
  } else if (code < 4) {
    if (code == 2)
      cancel<0, TAIL>(bk, st, rdlane(v.x, j), rdlane(u.w, j), u.z, j);
    else
      cancel<1, TAIL>(bk, st, rdlane(v.x, j), rdlane(u.w, j), u.z, j);
  } else if (code < 6) {
    const int Q = rdlane(u.w, j);
    __builtin_assume(Q > 0);
    const int rem = code == 4 ? match<1, TAIL, X, false>(bk, st, sg, 0, Q, v, j)
                              : match<0, TAIL, X, false>(bk, st, sg, INT_MAX, Q, v, j);
    if (rem > 0) st.market_discarded += (unsigned)rem;
  }
}

// Fair issue among the waves of a SIMD.  The instruction arbiter favours the oldest
// wave, so of several books sharing a SIMD one runs ahead and the last one ends
// alone, at one wave's speed.  With rank >= 0 a wave's priority rotates with time
// (an epoch of 2^13 ticks of the 100 MHz real-time counter, about 82 us), offset by
// its rank, so that each wave holds the highest priority a quarter of the time.
// Compiled in only where it runs (X bit 2): the code alone slows a lone wave.
__device__ __forceinline__ void rotate_priority(int rank) {
  const unsigned epoch = (unsigned)(__builtin_amdgcn_s_memrealtime() >> 13);
  switch ((epoch + (unsigned)rank) & 3) {
    case 0: __builtin_amdgcn_s_setprio(0); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    default: __builtin_amdgcn_s_setprio(3); break;
  }
}

// Record k0 + lane of a book's stream -- source 1 msgs[beg1, beg1 + n1), then
// source 2 (the step form's agent orders) msgs2[beg2, beg2 + n2) -- as u = (type,
// side, P, Q) and v = (OID, TID, Ts, Tns); zeros past the stream's end.
__device__ __forceinline__ void fetch_chunk(const ProcArgs &a, long long beg1, long long n1, long long beg2,
                                            long long total, long long k0, int4 &u, int4 &v) {
  const long long k = k0 + lane_id();
  if (k < total) {
    const int32_t *rec = k < n1 ? a.msgs + (beg1 + k) * kMsgFields : a.msgs2 + (beg2 + k - n1) * kMsgFields;
    const int4 *mp = reinterpret_cast<const int4 *>(rec);
    u = mp[0];
    v = mp[1];
  } else {
    u = v = make_int4(0, 0, 0, 0);
  }
}

// The book's messages in 64-message chunks, each loaded one chunk ahead of its use;
// (un, vn) is the first chunk, already requested by the caller.  Returns true, with
// the book's state abandoned, when a chunk shows the times going backwards in a form
// without the timed loop (kTimedInline).
template <bool TAIL, int X>
__device__ __forceinline__ bool process_all(Book &bk, RState &st, Stage &sg, const ProcArgs &a, long long beg1,
                                            long long n1, long long beg2, long long n2, int32_t *l2_rows, int4 un,
                                            int4 vn, int rank, int pk) {
  const int l = lane_id();
  const long long total = n1 + n2;
#pragma nounroll
  for (long long k0 = 0; k0 < total; k0 += kWave) {
    if constexpr ((X & 4) != 0) rotate_priority(rank);
    const int cnt = (int)((total - k0) < kWave ? (total - k0) : kWave);
    const int4 u = un, v = vn;
    if (k0 + kWave < total) fetch_chunk(a, beg1, n1, beg2, total, k0 + kWave, un, vn);
    const int T = u.x, S = u.y;
    const bool ok = (l < cnt) & (T >= 1) & (T <= 4) & ((S == 1) | (S == -1));
    // code 7 also for Q <= 0: such a cancel removes nothing and such a limit or
    // market order neither trades nor rests; only the counts and the time check see it
    const int code = !(ok & (u.w > 0)) ? 7 : (T == 1 ? 0 : T == 4 ? 4 : 2) + (S == 1 ? 1 : 0);
    const uint64_t vmask = ballot(ok);
    if (vmask) {
      // times of valid messages must not decrease: compare with the previous valid
      // lane, or with the last valid time before this chunk
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
      // submitted quantity of limit and market orders (Q > 0 only)
      const int qpos = u.w > 0 ? u.w : 0;
      sg.limit_qty += (unsigned)(code < 2 ? qpos : 0);
      sg.market_qty += (unsigned)((code >> 1) == 2 ? qpos : 0);
      sg.cancel_qty += (unsigned)((code >> 1) == 1 ? qpos : 0);
    }
    if constexpr ((X & 1) != 0 && kAgentMask<TAIL, X>) st.agm = ballot(v.y == st.agent_tid);
    // messages of this chunk that come from source 1 (they get per-message L2 rows)
    const int c1 = (int)(n1 - k0 < 0 ? 0 : (n1 - k0 < cnt ? n1 - k0 : cnt));
    if (LOB_LIKELY(!(st.flags & kFlagTimeOrder))) {
      int c = rdlane(code, 0);
#pragma nounroll
      for (int j = 0; j < cnt; ++j) {
        int cn = 0;
        if constexpr (kReadAhead<TAIL, X>)
          cn = rdlane(code, (j + 1) & (kWave - 1));
        else
          c = rdlane(code, j);
        process_msg<TAIL, X, false>(bk, st, sg, c, u, v, j, (int)k0 + j, pk);
        if constexpr ((X & 16) != 0) {
          if (j < c1) write_l1<TAIL>(bk, st, l2_rows + (k0 + j) * 4);  // (the host gives X bit 4 rows)
        } else if constexpr ((X & 2) != 0) {
          if (l2_rows && j < c1) write_l2<TAIL>(bk, st, a.levels, l2_rows + (k0 + j) * 4 * a.levels);
        }
        if constexpr (kReadAhead<TAIL, X>) c = cn;
      }
    } else if constexpr (kTimedInline<TAIL, X>) {
      // a book whose times went backwards: the same loop with the timed insert
#pragma nounroll
      for (int j = 0; j < cnt; ++j) {
        const int c = rdlane(code, j);
        process_msg<TAIL, X, true>(bk, st, sg, c, u, v, j, (int)k0 + j, pk);
        if constexpr ((X & 16) != 0) {
          if (j < c1) write_l1<TAIL>(bk, st, l2_rows + (k0 + j) * 4);
        }
      }
    } else {
      return true;
    }
    flush<TAIL, X>(st, sg, v);  // the staged records name messages of this chunk
  }
  return false;
}

// Slot s (< n) of one side of the loaded book: its P, Q, OID and handle.
template <bool FILLS>
__device__ __forceinline__ Chunk load_slot(const int2 *base, int cap, int s, int agent_tid) {
  const int2 pq = base[s], ot = base[cap + s];
  Chunk x;
  x.p = pq.x;
  x.q = pq.y;
  x.o = ot.x;
  x.h = (-1 - s) * 2 + ((FILLS && ot.y == agent_tid) ? 1 : 0);
  return x;
}

// Slots s (< n) of one side, zeros past the side's end.  FLAT: every lane loads (a
// lane past the end reads slot 0, which every book has) and a select drops what is
// not used; no load sits in a divergent branch, so the loads of all chunks are in
// flight together (used without a tail, where a call is often short; the TAIL
// form, short of scalar registers, keeps the branch).
template <bool FLAT>
__device__ __forceinline__ void load_chunk(Chunk &x, const int2 *base, int cap, int s, int n, int agent_tid,
                                           bool extra) {
  const bool in = s < n;
  if constexpr (FLAT) {
    const Chunk y = extra ? load_slot<true>(base, cap, in ? s : 0, agent_tid)
                          : load_slot<false>(base, cap, in ? s : 0, agent_tid);
    x.p = in ? y.p : 0;
    x.q = in ? y.q : 0;
    x.o = in ? y.o : 0;
    x.h = in ? y.h : 0;
  } else if (in) {
    x = extra ? load_slot<true>(base, cap, s, agent_tid) : load_slot<false>(base, cap, s, agent_tid);
  } else {
    x.p = x.q = x.o = x.h = 0;
  }
}


// TID, Ts, Tns of order x (one per lane), found through its handle in the stream
// or in the loaded side `src` (the other buffer, not written by this launch).
// FLAT: the two sources are chosen by address and every lane loads (a lane without
// an order, valid false, reads slot 0 of src), so that no load sits in a divergent
// branch; otherwise only valid lanes call it and each source has its own loads.
template <bool FLAT>
__device__ __forceinline__ int4 order_meta(const Chunk &x, bool valid, const int2 *src, int cap, const Streams &m) {
  long long idx = (!FLAT || valid) ? (x.h >> 1) : -1;
  if constexpr (FLAT) {
    const int32_t *pt;  // TID
    const int2 *ptt;    // (Ts, Tns)
    if (idx >= 0) {
      if (idx >= m.total) idx = m.total - 1;  // (cannot happen: a handle names a message of this stream)
      const int32_t *rec = idx < m.n1 ? m.msgs + (m.beg1 + idx) * kMsgFields
                                      : m.msgs2 + (m.beg2 + idx - m.n1) * kMsgFields;
      pt = rec + 5;
      ptt = reinterpret_cast<const int2 *>(rec + 6);
    } else {
      int os = (int)(-1 - idx);
      if (os >= cap) os = cap - 1;  // (cannot happen: a loaded slot is below the capacity)
      pt = reinterpret_cast<const int32_t *>(src + cap + os) + 1;
      ptt = src + 2 * cap + os;
    }
    const int t = *pt;
    const int2 tt = *ptt;
    return make_int4(t, tt.x, tt.y, 0);
  } else {
    int t, ts, tns;
    if (idx >= 0) {
      if (idx >= m.total) idx = m.total - 1;
      const int32_t *rec = idx < m.n1 ? m.msgs + (m.beg1 + idx) * kMsgFields
                                      : m.msgs2 + (m.beg2 + idx - m.n1) * kMsgFields;
      const int4 r = reinterpret_cast<const int4 *>(rec)[1];  // (OID, TID, Ts, Tns)
      t = r.y;
      ts = r.z;
      tns = r.w;
    } else {
      int os = (int)(-1 - idx);
      if (os >= cap) os = cap - 1;
      t = src[cap + os].y;
      const int2 tt = src[2 * cap + os];
      ts = tt.x;
      tns = tt.y;
    }
    return make_int4(t, ts, tns, 0);
  }
}

// Order x (one per lane) with its TID, Ts, Tns stored at slot s of one side of the
// written book `dst`.
__device__ __forceinline__ void put_order(const Chunk &x, const int4 &mt, int2 *dst, int cap, int s) {
  dst[s] = make_int2(x.p, x.q);
  dst[cap + s] = make_int2(x.o, mt.x);
  dst[2 * cap + s] = make_int2(mt.y, mt.z);
}

// The book goes to the LDS engine after this launch (kTimedInline): it is marked in
// its header; nothing of this launch's work on it is committed.
__device__ __forceinline__ void defer_book(BookHdr *h) {
  if (lane_id() == 0) h->deferred = 1;
}

// TAIL form: tails of the two sides in LDS at `lds`, a.W entries each.
template <bool TAIL, int X>
__device__ void run_book(const ProcArgs &a, int i, int2 *lds) {
  const int l = lane_id();
  const int book = a.book_ids ? uni(a.book_ids[i]) : i;
  if (book < 0 || book >= a.n_total) return;
  // the book's messages: msgs[beg1, beg1 + n1), then msgs2 (the step form's agent
  // orders) [i * w2, i * w2 + n2)
  long long beg1 = 0, n1 = 0;
  auto stream_range = [&]() {
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
  };
  const long long n2 = (a.msgs2 && a.w2 > 0) ? a.w2 : 0;
  // without a tail the first message chunk is requested before the book's header
  // and orders; the TAIL form, whose calls are long, requests it after them
  int4 u0, v0;
  if constexpr (!TAIL) {
    stream_range();
    fetch_chunk(a, beg1, n1, (long long)i * a.w2, n1 + n2, 0, u0, v0);
  }
  BookHdr *h = a.hdr + book;
  RState st;
  st.n[0] = uni(h->n[0]);
  st.n[1] = uni(h->n[1]);
  st.cap = uni(h->cap);
  if (st.cap > (TAIL ? kSlots + a.W : kSlots)) {  // not launched for such books; leave the book untouched
    if (l == 0) h->flags |= kFlagBadLoad;
    return;
  }
  st.flags = uni(h->flags);
  if constexpr (!kTimedInline<TAIL, X>) {
    if (LOB_UNLIKELY(st.flags & kFlagTimeOrder)) {
      defer_book(h);
      return;
    }
  }
  st.small_lim = st.cap < kWave ? st.cap : kWave;
  st.trades = st.misses = 0;
  st.cancel_short = st.market_discarded = st.rejected_qty = 0;
  st.last_ts = uni(h->last_ts);
  st.last_tns = uni(h->last_tns);
  st.seen = uni(h->seen_time);
  {
    const long long count = uni64(h->log_count), room = uni64(h->log_cap) - count;
    st.log = a.log ? a.log + (uni64(h->log_off) + count) * kTradeFields : nullptr;
    st.log_room = room < 0 ? 0 : (room > INT_MAX ? INT_MAX : (int)room);
    st.logged = 0;
  }
  const int row = a.out_rows ? uni(a.out_rows[i]) : i;  // output row of this book
  st.fills = a.fills ? a.fills + (int64_t)row * a.fill_cap * kTradeFields : nullptr;
  st.fill_cap = a.fill_cap;
  st.fill_count = 0;
  st.agent_tid = a.agent_tid;
  st.agm = 0;

  if constexpr (TAIL) stream_range();

  if (n1 + n2 >= (1LL << 30)) {  // handles hold message indices below 2^30
    if (l == 0) h->flags |= kFlagBadLoad;
    return;
  }

  // the loaded book, and the other buffer of this book, which receives the result
  const long long off = uni64(h->book_off);
  const long long off_out = off < a.books_half ? off + a.books_half : off - a.books_half;
  const int2 *hb = a.books + off;
  int2 *ob = a.books + off_out;
  const int cap = st.cap;
  Book bk;
  load_chunk<!TAIL>(bk.ask.c0, hb, cap, l, st.n[0], st.agent_tid, (X & 1) != 0);
  load_chunk<!TAIL>(bk.ask.c1, hb, cap, kWave + l, st.n[0], st.agent_tid, (X & 1) != 0);
  load_chunk<!TAIL>(bk.bid.c0, hb + 3 * (int64_t)cap, cap, l, st.n[1], st.agent_tid, (X & 1) != 0);
  load_chunk<!TAIL>(bk.bid.c1, hb + 3 * (int64_t)cap, cap, kWave + l, st.n[1], st.agent_tid, (X & 1) != 0);
  if constexpr (TAIL) {
    // slot s >= 128 of a side holding n orders is tail entry n - 1 - s
    for (int sd = 0; sd < 2; ++sd) {
      Tail &t = bk.tl[sd];
      t.a = reinterpret_cast<int4 *>(lds + sd * 2 * a.W);  // a.W int4 per side
      const int n = st.n[sd];
      const int2 *src = hb + (int64_t)sd * 3 * cap;
      for (int s = kSlots + l; s < n; s += kWave) tail_put(t, n - 1 - s, load_slot<(X & 1) != 0>(src, cap, s, st.agent_tid));
    }
  }
  Stage sg;
  sg.p = sg.q = sg.po = sg.j = 0;
  sg.k = 0;
  sg.limit_qty = sg.market_qty = sg.traded_qty = sg.cancel_qty = 0;

  // ragged launches raise the longest streams' waves for good; launches whose waves
  // share SIMDs (X bit 2) rotate priorities (rank: the wave's slot on its SIMD, bits
  // 3:0 of the HW_ID register)
  if (a.prio_len > 0 && n1 >= a.prio_len) __builtin_amdgcn_s_setprio(3);
  int rank = 0;
  if constexpr ((X & 4) != 0) rank = (int)(__builtin_amdgcn_s_getreg((3 << 11) | 4) & 3);
  // per-message L2 rows of source 1: contiguous by message index, or l2_stride
  // int32 apart per listed book
  int32_t *l2_rows = a.l2_mode != 1 ? nullptr
                     : a.l2_stride ? a.l2_out + (int64_t)i * a.l2_stride : a.l2_out + beg1 * 4 * a.levels;
  Origin g;
  g.m.msgs = a.msgs;
  g.m.msgs2 = a.msgs2;
  g.m.beg1 = beg1;
  g.m.n1 = n1;
  g.m.beg2 = (long long)i * a.w2;
  g.m.total = n1 + n2;
  g.hb = hb;
  g.cap = cap;
  if constexpr (TAIL) fetch_chunk(a, beg1, n1, (long long)i * a.w2, n1 + n2, 0, u0, v0);
  const bool went_back =
      process_all<TAIL, X>(bk, st, sg, a, beg1, n1, (long long)i * a.w2, n2, l2_rows, u0, v0, rank,
                           kTimedInline<TAIL, X> ? pack_origin(g) : 0);
  if (LOB_UNLIKELY(went_back)) {
    // nothing is committed yet: the header, and the buffer the book was loaded from,
    // are as they were, so the LDS engine takes this launch's stream from the start
    defer_book(h);
    return;
  }
  if (a.l2_mode == 2) write_l2<TAIL>(bk, st, a.levels, a.l2_out + (int64_t)row * 4 * a.levels);

  const Streams &ms = g.m;
  if constexpr (!TAIL) {
    // the orders' TID, Ts, Tns are all requested before any order is written (the
    // written buffer may alias the read ones as far as the compiler knows)
    int4 mt[2][2];
    for (int sd = 0; sd < 2; ++sd) {
      const Side &S = sd == 0 ? bk.ask : bk.bid;
      const int n = st.n[sd];
      const int2 *src = hb + (int64_t)sd * 3 * cap;
      mt[sd][0] = order_meta<true>(S.c0, l < n, src, cap, ms);
      mt[sd][1] = order_meta<true>(S.c1, kWave + l < n, src, cap, ms);
    }
    for (int sd = 0; sd < 2; ++sd) {
      const Side &S = sd == 0 ? bk.ask : bk.bid;
      const int n = st.n[sd];
      int2 *dst = ob + (int64_t)sd * 3 * cap;
      if (l < n) put_order(S.c0, mt[sd][0], dst, cap, l);
      if (kWave + l < n) put_order(S.c1, mt[sd][1], dst, cap, kWave + l);
    }
  } else {
    // long calls: the order of the loads does not matter; this form measured faster
    for (int sd = 0; sd < 2; ++sd) {
      const Side &S = sd == 0 ? bk.ask : bk.bid;
      const int n = st.n[sd];
      const int2 *src = hb + (int64_t)sd * 3 * cap;
      int2 *dst = ob + (int64_t)sd * 3 * cap;
      if (l < n) put_order(S.c0, order_meta<false>(S.c0, true, src, cap, ms), dst, cap, l);
      if (kWave + l < n) put_order(S.c1, order_meta<false>(S.c1, true, src, cap, ms), dst, cap, kWave + l);
      for (int s = kSlots + l; s < n; s += kWave) {
        const Chunk x = tail_get(bk.tl[sd], n - 1 - s);
        put_order(x, order_meta<false>(x, true, src, cap, ms), dst, cap, s);
      }
    }
  }
  if (st.fills) {
    if (st.fill_count > st.fill_cap) st.flags |= kFlagFillsFull;
    if (l == 0 && a.fill_counts) a.fill_counts[row] = st.fill_count;
  }
  const long long limit_qty = wave_sum64(sg.limit_qty), market_qty = wave_sum64(sg.market_qty),
                  traded_qty = wave_sum64(sg.traded_qty);
  const long long cancelled_qty = wave_sum64(sg.cancel_qty) - st.cancel_short;
  if (l == 0) {
    h->book_off = off_out;
    h->n[0] = st.n[0];
    h->n[1] = st.n[1];
    h->flags = st.flags;
    h->n_msgs += n1 + n2;
    h->n_trades += st.trades;
    h->limit_qty += limit_qty;
    h->market_qty += market_qty;
    h->traded_qty += traded_qty;
    h->cancelled_qty += cancelled_qty;
    h->market_discarded += st.market_discarded;
    h->rejected_qty += st.rejected_qty;
    h->cancel_miss += st.misses;
    h->last_ts = st.last_ts;
    h->last_tns = st.last_tns;
    h->seen_time = st.seen;
    h->log_count += st.logged;
  }
}

template <bool TAIL, int X>
__global__ void __launch_bounds__(1024) k_process_small(ProcArgs a) {
  extern __shared__ __align__(16) int2 tail_smem[];
  const int w = uni(threadIdx.x / kWave);  // uniform: one wave = one book
  const int i = blockIdx.x * a.bpb + w;
  if (i >= a.n) return;
  run_book<TAIL, X>(a, i, TAIL ? tail_smem + (int64_t)w * a.lds_int2_per_wave : nullptr);
}

__global__ void k_selftest_shift(int32_t *out) {
  const int l = lane_id();
  const int x = 3 * l + 1;
  out[l] = shr1(x, -5);        // lane l-1; lane 0 gets the fill
  out[64 + l] = shl1(x, -7);   // lane l+1; lane 63 gets the fill
  out[128 + l] = from_lane(x, (l + 5) & 63);
  out[192 + l] = up1(x);         // lane l-1; lane 0 gets 0
  out[256 + l] = dn1(x);         // lane l+1; lane 63 gets 0
  out[320 + l] = wl(x, -9, 17);  // lane 17 replaced
}

}  // namespace

int small_book_slots() { return kSlots; }

// tail = false: books of capacity <= 128; tail = true: a.W tail entries per side in
// LDS (a.lds_int2_per_wave = 4 * a.W per wave)
// X of the instantiation a launch runs: bit 0 agent fills, bit 1 per-message L2, bit
// 2 rotating priorities (without a tail only), bit 3 the TAIL form's chunk-0 insert
// (kChunk0Insert; alone only), bit 4 per-message rows of level 1 (with agent fills:
// the execution step)
static int small_form(const ProcArgs &a, bool tail) {
  int x = (a.fills != nullptr ? 1 : 0) | (a.l2_mode == 1 ? 2 : 0) | (!tail && a.rotate ? 4 : 0);
  if (tail && x == 0 && a.tail_shallow) x = 8;
  if ((x & 3) == 3 && a.levels == 1 && a.l2_out != nullptr) x |= 16;
  return x;
}

bool small_defers(const ProcArgs &a, bool tail) {
  const int x = small_form(a, tail);
  return tail || ((x & 2) != 0 && (x & 16) == 0);  // not kTimedInline
}

hipError_t launch_process_small(const ProcArgs &a, bool tail, hipStream_t s) {
  const int threads = a.bpb * kWave;
  const int grid = (a.n + a.bpb - 1) / a.bpb;
  const size_t lds = tail ? (size_t)a.bpb * a.lds_int2_per_wave * sizeof(int2) : 0;
  const int x = small_form(a, tail);
  switch ((tail ? 32 : 0) | x) {
#define LOB_SMALL_CASE(T, X)                                                                   \
  case (T ? 32 : 0) | X:                                                                       \
    hipLaunchKernelGGL((k_process_small<T, X>), dim3(grid), dim3(threads), T ? lds : 0, s, a); \
    break;
    LOB_SMALL_CASE(false, 0)
    LOB_SMALL_CASE(false, 1)
    LOB_SMALL_CASE(false, 2)
    LOB_SMALL_CASE(false, 3)
    LOB_SMALL_CASE(false, 4)
    LOB_SMALL_CASE(false, 5)
    LOB_SMALL_CASE(false, 6)
    LOB_SMALL_CASE(false, 7)
    LOB_SMALL_CASE(false, 19)
    LOB_SMALL_CASE(false, 23)
    LOB_SMALL_CASE(true, 0)
    LOB_SMALL_CASE(true, 1)
    LOB_SMALL_CASE(true, 2)
    LOB_SMALL_CASE(true, 3)
    LOB_SMALL_CASE(true, 19)
    LOB_SMALL_CASE(true, 8)
#undef LOB_SMALL_CASE
  }
  return hipGetLastError();
}

hipError_t set_process_small_lds_limit(size_t bytes) {
  const void *k[6] = {(const void *)k_process_small<true, 0>, (const void *)k_process_small<true, 1>,
                      (const void *)k_process_small<true, 2>, (const void *)k_process_small<true, 3>,
                      (const void *)k_process_small<true, 8>, (const void *)k_process_small<true, 19>};
  for (const void *f : k) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_selftest_shift(int32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_selftest_shift, dim3(1), dim3(64), 0, s, out);
  return hipGetLastError();
}

}  // namespace lob
