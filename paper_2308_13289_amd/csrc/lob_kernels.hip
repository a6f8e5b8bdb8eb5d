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

#include <algorithm>
#include <limits.h>
#include <stdint.h>

#include "lob_device.h"
#include "lob_internal.h"
#include "lob_lds_engine.h"

namespace lob {
namespace {

using namespace dev;
using lds::run_book;
using lds::View;
using lds::write_l2;

template <bool SPILL>
__global__ void __launch_bounds__(1024) k_process(ProcArgs a) {
  extern __shared__ int2 smem[];
  const int w = uni(threadIdx.x / kWave);  // uniform: one wave = one book
  const int i = blockIdx.x * a.bpb + w;
  if (i >= a.n) return;
  int2 *lds = smem + (int64_t)w * a.lds_int2_per_wave;
  run_book<SPILL>(a, i, lds, a.W);
}

// The books of a launch that the register kernel left to this engine (times went
// backwards; marked `deferred` in their headers): the waves scan the listed books 64
// at a time and run the whole of the launch's stream for each marked one, with a
// window of W slots per side in LDS and the rest in HBM.
__global__ void __launch_bounds__(256) k_process_deferred(ProcArgs a, int W) {
  extern __shared__ int2 dsmem[];
  const int l = lane_id();
  const int w = uni(threadIdx.x / kWave);
  const int waves = gridDim.x * (blockDim.x / kWave);
  int2 *lds = dsmem + (int64_t)w * 6 * W;
  for (int base = (blockIdx.x * (blockDim.x / kWave) + w) * kWave; base < a.n; base += waves * kWave) {
    const int k = base + l;
    bool marked = false;
    if (k < a.n) {
      const int b = a.book_ids ? a.book_ids[k] : k;
      marked = b >= 0 && b < a.n_total && a.hdr[b].deferred != 0;
    }
    for (uint64_t m = ballot(marked); m; m &= m - 1) {
      const int i = base + first_set(m);
      run_book<true>(a, i, lds, W);
      if (l == 0) a.hdr[a.book_ids ? a.book_ids[i] : i].deferred = 0;
    }
  }
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
  h->deferred = 0;
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
  write_l2(B, st, L, out + (int64_t)i * 4 * L);
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
// Rows out of priority order (prices, or times at one price) or past the capacity
// flag the book; the header's latest time becomes at least the newest order's.
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
  // the latest (Ts, Tns) among the written orders, as one ordered key per lane
  long long newest = LLONG_MIN;
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
        // priority order: prices ordered, equal prices by time (equal times keep
        // the written order, which stands for arrival)
        if (s > 0)
          unsorted = (sd == 0 ? r[0] < r[-6] : r[0] > r[-6]) ||
                     (r[0] == r[-6] && (r[4] < r[-2] || (r[4] == r[-2] && r[5] < r[-1])));
        const long long key = ((long long)r[4] << 32) | (unsigned)(r[5] ^ INT_MIN);
        newest = key > newest ? key : newest;
      }
      if (ballot(unsorted)) bad = 1;
    }
    if (l == 0) h->n[sd] = live;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    const long long other = ((long long)__shfl_xor((int)(newest >> 32), o, kWave) << 32) |
                            (unsigned)__shfl_xor((int)(unsigned)newest, o, kWave);
    newest = other > newest ? other : newest;
  }
  if (l == 0) {
    if (bad) h->flags |= kFlagBadLoad;
    // the book's latest time is at least that of every written order, so that a later
    // message stamped before one of them counts as time going backwards
    if (newest != LLONG_MIN) {
      const int ts = (int)(newest >> 32), tns = (int)(unsigned)newest ^ INT_MIN;
      if (!h->seen_time || ts > h->last_ts || (ts == h->last_ts && tns > h->last_tns)) {
        h->last_ts = ts;
        h->last_tns = tns;
      }
      h->seen_time = 1;
    }
  }
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
    // the initial orders' time is the book's latest time: a later message stamped
    // before it counts as time going backwards
    h->last_ts = ts;
    h->last_tns = tns;
    h->seen_time = 1;
    h->deferred = 0;
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

// After a register-kernel launch that may leave books to the LDS engine: up to 64
// blocks of 4 waves, W slots per side in LDS.
hipError_t launch_process_deferred(const ProcArgs &a, int W, hipStream_t s) {
  const int blocks = std::max(1, std::min(64, (a.n + 4 * kWave - 1) / (4 * kWave)));
  hipLaunchKernelGGL(k_process_deferred, dim3(blocks), dim3(256), (size_t)4 * 6 * W * sizeof(int2), s, a, W);
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
