// lob_internal.h -- device-side layout shared by the kernels and the host code of liblob.
//
// Device memory of a context:
//   hdr   [n_books] BookHdr           counters, live counts, where the book's arrays are
//   books [2][sum 6*cap] int2         per book, per side s (0 asks, 1 bids), three pair
//                                     arrays of `cap` entries each, kept in price-time
//                                     priority (slot 0 = best):  (P, Q), (OID, TID),
//                                     (Ts, Tns)  -- the six order features of the paper's
//                                     Section 4, two per 8-byte word.  Two buffers per
//                                     book, `books_half` int2 apart: the header's
//                                     book_off names the current one; the register
//                                     kernel writes its result to the other and
//                                     switches book_off, the other kernels work in place
//   log   [sum log_cap][6] int32      per book, the trade records not yet read
#pragma once
#include <stdint.h>

namespace lob {

constexpr int kWave = 64;
constexpr int kMsgFields = 8;
constexpr int kTradeFields = 6;

// flags (same values as LOB_BOOK_* in lob.h)
constexpr int kFlagSideFull = 1;
constexpr int kFlagTimeOrder = 2;
constexpr int kFlagTradeFull = 4;
constexpr int kFlagFillsFull = 8;
constexpr int kFlagBadLoad = 16;

struct alignas(16) BookHdr {
  int32_t n[2];  // live orders: [0] asks, [1] bids
  int32_t cap;   // capacity per side
  int32_t flags;
  int64_t book_off;   // first int2 of this book's current arrays in `books`
  int64_t log_off;    // first record of this book's trade log
  int64_t log_cap;    // records the log can hold
  int64_t log_count;  // records waiting in the log
  int64_t n_msgs, n_trades, limit_qty, market_qty, traded_qty, cancelled_qty, market_discarded,
      rejected_qty, cancel_miss;
  int32_t last_ts, last_tns;  // time of the last processed message
  int32_t seen_time;          // 1 once a message with a valid type was processed
  int32_t deferred;           // 1: left by the register kernel to k_process_deferred
  int32_t pad[2];
};
static_assert(sizeof(BookHdr) == 144, "BookHdr layout");

// Arguments of the matching kernels (passed by value).
struct ProcArgs {
  BookHdr *hdr;
  int2 *books;
  int64_t books_half;  // int2 between a book's two buffers
  int32_t *log;        // trade log base, or nullptr: do not log trades
  const int32_t *book_ids;  // nullptr: listed book i is book i
  int32_t n;                // listed books
  int32_t n_total;          // books in the context (ids outside [0, n_total) are skipped)
  // message source 1: msgs[offs[i] .. offs[i+1]) or, when offs == nullptr, msgs[i*w1 .. (i+1)*w1)
  const int32_t *msgs;
  const int64_t *offs;
  int32_t w1;
  // message source 2 (step actions): msgs2[i*w2 .. (i+1)*w2)
  const int32_t *msgs2;
  int32_t w2;
  int32_t l2_mode;     // 0 none, 1 per message (indexed like source 1), 2 final (per listed book)
  int32_t levels;
  int32_t *l2_out;
  int64_t l2_stride;   // l2_mode 1: 0 = rows by source-1 message index; else listed book i's
                       // rows start at l2_out + i * l2_stride (int32 elements)
  // agent fills (step form)
  int32_t *fills;      // [n][fill_cap][6] or nullptr
  int32_t fill_cap;
  int32_t *fill_counts;
  int32_t agent_tid;
  // LDS window
  int32_t W;           // LDS slots per side-pair array
  int32_t bpb;         // books (waves) per block
  int32_t lds_int2_per_wave;
  // explicit per-book message ranges ([n][2] begin, end into msgs) and output rows
  // (L2 / fills row of listed book i); nullptr = offs / identity
  const int64_t *ranges;
  const int32_t *out_rows;
  // a wave whose book has at least this many source-1 messages raises its issue
  // priority (0: none); ragged calls set it so the longest streams, the critical
  // path, are not slowed by the short ones sharing their compute unit
  int64_t prio_len;
  // 1: with prio_len 0, the register kernel's waves rotate their issue priority
  // (set by the host when a launch has more books than the GPU has SIMDs, so that
  // waves share SIMDs)
  int32_t rotate;
  // 1: launches of the TAIL form without agent fills and per-message L2 take the
  // instantiation laid out for sides of fewer than 64 orders (plan.tail_shallow)
  int32_t tail_shallow;
};

}  // namespace lob
