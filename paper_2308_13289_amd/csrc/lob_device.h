// lob_device.h -- wavefront primitives and per-book state shared by the matching
// kernels (lob_kernels.hip: book sides in LDS; lob_small.hip: books of capacity
// <= 128 wholly in registers).
#pragma once
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include "lob_internal.h"

namespace lob {
namespace dev {

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }
// The lane id as an opaque value: address arithmetic built on it is recomputed where
// it is used instead of being hoisted out of the message loop into a VGPR per site.
__device__ __forceinline__ int lane_id_local() {
  int x;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(x));
  return x;
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ int popc(uint64_t m) { return __builtin_popcountll(m); }
__device__ __forceinline__ int first_set(uint64_t m) { return __builtin_ctzll(m); }
__device__ __forceinline__ int rdlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uni64(long long v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v & 0xffffffffll));
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
// lanes 0..lane inclusive
__device__ __forceinline__ uint64_t mask_le() { return ~0ull >> (63 - lane_id()); }
__device__ __forceinline__ uint64_t mask_lt() { return mask_le() >> 1; }

// Inclusive prefix sum over the 64 lanes: four row_shr steps inside each row of 16
// lanes, then row_bcast:15 and row_bcast:31 carry the row totals upwards.
__device__ __forceinline__ int scan_incl(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false); // row_bcast:15 -> rows 1,3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false); // row_bcast:31 -> rows 2,3
  return x;
}

// The same scan of non-negative values with saturating adds: lane l receives
// min(x_0 + ... + x_l, INT_MAX) exactly, whatever the sum.
__device__ __forceinline__ int sat_add(int a, int b) { return __builtin_elementwise_add_sat(a, b); }
__device__ __forceinline__ int scan_incl_sat(int x) {
  x = sat_add(x, __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true));
  x = sat_add(x, __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true));
  x = sat_add(x, __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true));
  x = sat_add(x, __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true));
  x = sat_add(x, __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false));
  x = sat_add(x, __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false));
  return x;
}

// Quantities below this bound take the matching scan's exact int32 form: each
// resting quantity clamped to q + 1 decides every fill test as the true value does,
// and 64 such values sum below 2^31.
constexpr int kScanExactQ = 1 << 24;

// Whole-wave shifts by one lane (DPP wave_shr:1 / wave_shl:1): lane l receives
// lane l-1 (shr) or l+1 (shl); the lane with no source (0, resp. 63) receives `fill`.
__device__ __forceinline__ int shr1(int x, int fill) {
  return __builtin_amdgcn_update_dpp(fill, x, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int shl1(int x, int fill) {
  return __builtin_amdgcn_update_dpp(fill, x, 0x130, 0xf, 0xf, false);
}
// Value of x in lane `src` (0..63) for every lane.
__device__ __forceinline__ int from_lane(int x, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, x); }

// L2 level quantities over one 64-slot chunk of a side taken in priority order.  q:
// the slot's quantity (0 past the side's end); ml: ballot of the slots that end a
// level.  A level's quantity is summed exactly and reported as min(sum, INT_MAX)
// (the L2 record is int32).  Returns that quantity on the lanes of ml; carry (uniform)
// is the exact quantity of the level left open by the chunks before and becomes the
// one left open after this chunk.  Quantities below 2^25 sum in one int32 scan; a
// chunk holding a larger one sums its 16-bit halves separately.
__device__ __forceinline__ int level_qty(int q, uint64_t ml, long long &carry) {
  const uint64_t below = ml & mask_lt();
  const int src = below ? 63 - __builtin_clzll(below) : 0;
  const int last = ml ? 63 - __builtin_clzll(ml) : 0;
  int res;
  if (__builtin_expect(ballot(q >= (1 << 25)) == 0, 1)) {
    const int loc = scan_incl(q);
    const int prev = from_lane(loc, src);
    const int cc = carry > INT_MAX ? INT_MAX : (int)carry;
    res = below ? loc - prev : sat_add(cc, loc);
    const int tot = rdlane(loc, 63);
    carry = ml ? (long long)(tot - rdlane(loc, last)) : carry + tot;
  } else {
    const int lo = scan_incl(q & 0xffff), hi = scan_incl((int)((unsigned)q >> 16));
    const long long loc = ((long long)hi << 16) + lo;
    const long long prev = ((long long)from_lane(hi, src) << 16) + from_lane(lo, src);
    const long long v = below ? loc - prev : carry + loc;
    res = v > INT_MAX ? INT_MAX : (int)v;
    const long long tot = ((long long)rdlane(hi, 63) << 16) + rdlane(lo, 63);
    const long long at_last = ((long long)rdlane(hi, last) << 16) + rdlane(lo, last);
    carry = ml ? tot - at_last : carry + tot;
  }
  return res;
}

// Wave-uniform state of the book being processed.
struct State {
  int n[2];
  int cap, flags;
  long long n_msgs, n_trades, limit_qty, market_qty, traded_qty, cancelled_qty, market_discarded,
      rejected_qty, cancel_miss;
  int last_ts, last_tns, seen;
  int32_t *log;        // this book's log segment, or nullptr
  long long log_count, log_cap;
  int32_t *fills;      // this book's fills row, or nullptr
  int fill_cap, fill_count, agent_tid;
  int bP[2], bQ[2], bO[2], bT[2];  // slot 0 of each side (valid while n > 0)
};

// Store the fills of one matching chunk (lanes with `takes` form the prefix
// [0, ntr)) to the trade log and, when the book collects them, to the agent fills.
__device__ __forceinline__ void emit(State &st, bool takes, int ntr, int P, int fill, int pas_oid,
                                     int agg_oid, int ts, int tns, int pas_tid, int agg_tid) {
  const int l = lane_id();
  if (st.log) {
    const long long room = st.log_cap - st.log_count;
    if (takes && l < room) {
      int2 *r = reinterpret_cast<int2 *>(st.log + (st.log_count + l) * kTradeFields);
      r[0] = make_int2(P, fill);
      r[1] = make_int2(pas_oid, agg_oid);
      r[2] = make_int2(ts, tns);
    }
    const long long stored = room < ntr ? (room > 0 ? room : 0) : ntr;
    if (stored < ntr) st.flags |= kFlagTradeFull;
    st.log_count += stored;
  }
  if (st.fills) {
    const bool ag = takes && (pas_tid == st.agent_tid || agg_tid == st.agent_tid);
    const uint64_t ma = ballot(ag);
    if (ma) {
      const int k = st.fill_count + popc(ma & mask_lt());
      if (ag && k < st.fill_cap) {
        int2 *r = reinterpret_cast<int2 *>(st.fills + (int64_t)k * kTradeFields);
        r[0] = make_int2(P, fill);
        r[1] = make_int2(pas_oid, agg_oid);
        r[2] = make_int2(ts, tns);
      }
      st.fill_count += popc(ma);
    }
  }
}

// One trade from scalar values (lane 0 writes it).
__device__ __forceinline__ void emit_one(State &st, int P, int fill, int pas_oid, int agg_oid, int ts, int tns,
                                         int pas_tid, int agg_tid) {
  const bool lead = lane_id() == 0;
  if (st.log) {
    if (st.log_count < st.log_cap) {
      if (lead) {
        int2 *r = reinterpret_cast<int2 *>(st.log + st.log_count * kTradeFields);
        r[0] = make_int2(P, fill);
        r[1] = make_int2(pas_oid, agg_oid);
        r[2] = make_int2(ts, tns);
      }
      st.log_count++;
    } else {
      st.flags |= kFlagTradeFull;
    }
  }
  if (st.fills && (pas_tid == st.agent_tid || agg_tid == st.agent_tid)) {
    if (st.fill_count < st.fill_cap && lead) {
      int2 *r = reinterpret_cast<int2 *>(st.fills + (int64_t)st.fill_count * kTradeFields);
      r[0] = make_int2(P, fill);
      r[1] = make_int2(pas_oid, agg_oid);
      r[2] = make_int2(ts, tns);
    }
    st.fill_count++;
  }
}

}  // namespace dev
}  // namespace lob
