/*
 * lob_oracle.h -- reference oracle for the batched limit-order-book matcher.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this library.  The product path
 * (the HIP library and its binding) never links, loads or includes anything here,
 * and nothing here includes anything from the product path.
 *
 * What it computes: the sequential price-time-priority matching engine of
 * JAX-LOB (Frey et al. 2023), written out the way Section 4 states it:
 *   - a book side is a fixed-capacity, UNSORTED array of N orders
 *     o_i = [P, Q, OID, TID, Ts, Tns]; an empty position has every field -1
 *     (Section 4, eq. "features");
 *   - three basic operations, each followed by the clean-up that empties every
 *     order whose Q <= 0 (Section 4.1);
 *   - the best standing order found by a full scan every time it is needed
 *     (Section 4.1, eq. "best_price"), and the matching while-loop with inclusive
 *     price overlap (Section 4.1);
 *   - dispatch on the message type and side (Section 4.2);
 *   - cancellation of L2-snapshot initial orders by price (Section 5.1.1).
 * Every reading taken where the paper is silent or garbled is listed in the
 * comments of lob_oracle.c at the place it applies.
 *
 * Layouts (all int32 unless stated):
 *   message  : {type, side, price, qty, order_id, trader_id, time_s, time_ns}
 *              (the paper orders the fields [T, S, Q, P, OID, TID, Ts, Tns];
 *               this engine stores price before qty)
 *   trade    : {price, qty, passive_id, aggressive_id, time_s, time_ns,
 *               passive_trader_id, aggressive_trader_id}     (ORC_TRADE_FIELDS)
 *              The first six are the trade record of Section 4.1 (eq. "trade")
 *              with the standing order's id before the aggressor's; the last two
 *              let callers pick out fills that involve a given trader.
 *   L2       : [2][levels][2] = {asks, bids} x level x {price, qty}; a missing
 *              level is (-1, 0); a level's quantity is its exact sum capped at
 *              INT32_MAX (R19 in lob_oracle.c).
 *   book dump: [cap][6] per side in priority order, unused rows all -1.
 */
#ifndef LOB_ORACLE_H
#define LOB_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MSG_FIELDS 8
#define ORC_TRADE_FIELDS 8
#define ORC_ORDER_FIELDS 6

/* per-book flags */
#define ORC_FLAG_SIDE_FULL 1   /* a limit remainder was rejected: its side was full */
#define ORC_FLAG_TIME_ORDER 2  /* a message's time was earlier than the previous one */
#define ORC_FLAG_TRADE_FULL 4  /* the caller's trade buffer for this book overflowed */
#define ORC_FLAG_BAD_LOAD 16   /* an L2 snapshot handed to orc_seed_l2 was not a book */

/* L2 snapshot modes of orc_run */
#define ORC_L2_NONE 0
#define ORC_L2_PER_MESSAGE 1
#define ORC_L2_FINAL 2

typedef struct {
  int64_t n_msgs;            /* messages handed to the book (all types)          */
  int64_t n_trades;          /* trades generated (also those not stored)          */
  int64_t limit_qty;         /* sum of Q over limit messages with Q > 0           */
  int64_t market_qty;        /* sum of Q over market messages with Q > 0          */
  int64_t traded_qty;        /* sum of trade quantities                           */
  int64_t cancelled_qty;     /* quantity removed by cancel / delete               */
  int64_t market_discarded;  /* unmatched remainder of market orders              */
  int64_t rejected_qty;      /* limit remainder that found its side full          */
  int64_t cancel_miss;       /* cancels that found no order                       */
  int32_t flags;             /* ORC_FLAG_*                                        */
  int32_t pad;
} orc_stats;

typedef struct orc_book orc_book;

/* A book with capacity N per side, both sides empty.  NULL on bad N / no memory. */
orc_book *orc_new(int32_t N);
void orc_free(orc_book *b);

/* Process one message.  Trades are appended to `trades` (room for `max_trades`
 * records of ORC_TRADE_FIELDS); the number generated is returned (records beyond
 * max_trades are counted, not stored).  A message can generate at most N trades. */
int32_t orc_process(orc_book *b, const int32_t *msg, int32_t *trades, int32_t max_trades);

/* Top `levels` price levels per side into out[2][levels][2]. */
void orc_l2(const orc_book *b, int32_t levels, int32_t *out);

/* Live orders of a side (+1 bids, -1 asks) in priority order into out[N][6];
 * rows past the live ones are -1.  Returns the number of live orders. */
int32_t orc_dump(const orc_book *b, int32_t side, int32_t *out);

void orc_get_stats(const orc_book *b, orc_stats *out);
int32_t orc_capacity(const orc_book *b);

/* Initialise a book from an L2 snapshot (Section 5.1.1): l2 = [2][levels][2], side
 * 0 asks (best first, ascending prices), side 1 bids (best first, descending), each
 * entry (price, qty); entries with qty <= 0 are missing levels.  The book is
 * emptied and its counters cleared, then every present level becomes one order
 * holding the level's quantity, with trader id `tid` and time (ts, tns), which also
 * becomes the book's latest time for the time-order check.  Order ids
 * start at -9000 and descend, level by level, ask before bid (R14).  A snapshot
 * that is not a book -- prices not strictly ordered, bid >= ask, or more levels
 * than the capacity on a side -- leaves the book empty, sets ORC_FLAG_BAD_LOAD and
 * returns -1; otherwise returns the number of orders placed. */
int32_t orc_seed_l2(orc_book *b, const int32_t *l2, int32_t levels, int32_t tid, int32_t ts, int32_t tns);

/* Batch runner: books run independently on `n_threads` host threads.
 *   caps[n_books]            capacity per side of each book
 *   msgs[..][8], offs[n+1]   book i processes msgs[offs[i] .. offs[i+1])
 *   l2_mode, levels          ORC_L2_*; l2_out is [offs[n]][2][levels][2] for
 *                            PER_MESSAGE and [n][2][levels][2] for FINAL
 *   trades, trade_offs[n+1]  book i may store trade_offs[i+1]-trade_offs[i]
 *                            records from trades + trade_offs[i]*8 (may be NULL)
 *   trade_msg                NULL or int64 parallel to `trades`: index (into msgs)
 *                            of the message that produced each stored trade
 *   trade_counts[n]          trades generated per book (may be NULL)
 *   stats[n]                 per-book counters (may be NULL)
 *   dumps                    NULL or [n][2][maxcap][6]: final books, {asks, bids}
 *   dump_cap                 maxcap for `dumps`
 * Returns 0, or -1 on bad arguments / no memory. */
int32_t orc_run(int32_t n_books, const int32_t *caps, const int32_t *msgs,
                const int64_t *offs, int32_t l2_mode, int32_t levels, int32_t *l2_out,
                int32_t *trades, const int64_t *trade_offs, int64_t *trade_msg,
                int64_t *trade_counts, orc_stats *stats, int32_t *dumps, int32_t dump_cap,
                int32_t n_threads);

#ifdef __cplusplus
}
#endif
#endif
