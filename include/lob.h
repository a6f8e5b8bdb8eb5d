/*
 * lob.h -- C ABI of the MI355X (gfx950) batched limit-order-book matcher.
 *
 * Many independent limit order books are processed at once; inside a book every
 * message is processed strictly in order (JAX-LOB, Frey et al. 2023, Section 4.3:
 * message processing in a continuous double auction is serial, parallelism comes
 * from running many books side by side).  One GPU wavefront owns one book while
 * it runs.
 *
 * Conventions for every entry point:
 *   - Buffers are DEVICE pointers (e.g. a torch tensor's data_ptr() on the context's
 *     device) unless the name ends in _host.  They are owned by the caller and must
 *     stay valid until the stream reaches the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Calls
 *     enqueue work and return without waiting for the device unless stated.
 *   - Argument errors are reported synchronously as a negative lob_status and no
 *     work is enqueued; lob_last_error() then describes the error.  Conditions
 *     that depend on the data (a full side, an unknown order id, a full trade log,
 *     times going backwards) never fail a call: they are counted per book and
 *     read with lob_read_status.
 *   - A context is used by one host thread at a time.  A book id may appear at
 *     most once in one call; calls on one stream are processed in order.  Book ids
 *     in device arrays outside [0, n_books) are skipped.
 *   - Every field of every record is int32: prices in ticks, quantities in shares,
 *     ids, and times split into whole seconds and nanoseconds (Section 4.2).
 *
 * Records:
 *   message (8 x int32)  {type, side, price, qty, order_id, trader_id, time_s, time_ns}
 *       The fields of the paper's message m = [T, S, Q, P, OID, TID, Ts, Tns]
 *       (Section 4.2, eq. "message") with price stored before qty.  type: 1 limit,
 *       2 cancel, 3 delete, 4 market; any other type is skipped (zero padding,
 *       Section 5.1.1).  side: +1 bid (buy), -1 ask (sell); any other side is
 *       skipped.  price is ignored for market orders.  Times are expected not to
 *       decrease within a book; a decrease is flagged (LOB_BOOK_TIME_ORDER) and
 *       the results stay exact: priority among equal prices always follows the
 *       time stamps (Section 4.1), equal times keep arrival order.
 *   trade (6 x int32)    {price, qty, passive_id, aggressive_id, time_s, time_ns}
 *       The trade t_j of Section 4.1 (eq. "trade"): the standing order's price,
 *       the traded quantity, both order ids (standing first) and the aggressor's
 *       time.
 *   L2 snapshot          int32 [2][levels][2] = {asks, bids} x level x {price, qty}
 *       Distinct prices best first (asks ascending, bids descending) with the
 *       summed quantity of the orders at that price, summed exactly and reported
 *       as min(sum, INT32_MAX) (the record is int32); a missing level is (-1, 0).
 *   book dump            int32 [2][dump_cap][6] = {asks, bids} x order x
 *       {P, Q, OID, TID, Ts, Tns} (Section 4, eq. "features") in price-time
 *       priority; unused rows are -1 (the paper's empty marker).
 *
 * Matching (Section 4.1 and 4.2): a limit order is matched against the opposite
 * side while that side is non-empty, its remaining quantity is positive and the
 * best standing price overlaps its own (inclusive); each match trades
 * min(remaining, standing) at the standing price; the remainder rests as one new
 * order, or is rejected and counted when its side already holds `capacity`
 * orders.  A market order matches with price 0 (sell) or INT32_MAX (buy) and its
 * remainder is dropped.  Cancel and delete subtract their quantity from the order
 * with that id on the message's side (or, if there is none, from the best-priority
 * initial order -- id <= -9000 -- at the message's price, Section 5.1.1) and remove
 * it once its quantity is <= 0; a quantity <= 0 does nothing.  The best standing
 * order is the lowest ask / highest bid, earliest (Ts, Tns) first, then earliest
 * arrival (eq. "best_price" and the text before it).
 *
 * Input domain: every int32 value of every field.  Quantities are int32 shares
 * (Section 4.2); matching, cancels and trades are exact for any of them, including
 * sweeps whose fills add up past INT32_MAX, and the counters of lob_book_status
 * are int64.  Only an L2 level's summed quantity is capped (see above).
 */
#ifndef LOB_H
#define LOB_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lob_status;
#define LOB_OK 0
#define LOB_EINVAL (-1)   /* bad argument                                        */
#define LOB_ENOMEM (-2)   /* device or host allocation failed                    */
#define LOB_EDEVICE (-3)  /* a HIP call failed (message in lob_last_error)       */
#define LOB_ECAP (-6)     /* a size exceeds what the context was created for     */

#define LOB_MAX_CAPACITY 4096 /* orders per side per book                        */
#define LOB_MAX_LEVELS 64     /* L2 depth                                        */

/* l2_mode of lob_process_messages */
#define LOB_L2_NONE 0
#define LOB_L2_PER_MESSAGE 1 /* l2_out row k = snapshot after message k of msgs   */
#define LOB_L2_FINAL 2       /* l2_out row i = snapshot after listed book i's last */

/* per-book status flags (lob_book_status.flags) */
#define LOB_BOOK_SIDE_FULL 1    /* a limit remainder was rejected: side full     */
#define LOB_BOOK_TIME_ORDER 2   /* a message's time was earlier than the last one */
#define LOB_BOOK_TRADE_FULL 4   /* trades were dropped: the book's trade log full */
#define LOB_BOOK_FILLS_FULL 8   /* agent fills were dropped: the fills buffer full */
#define LOB_BOOK_BAD_LOAD 16    /* lob_write_book rows out of priority order or past
                                   the capacity, lob_seed_l2 given a snapshot that
                                   is not a book, or a call of the register kernel
                                   with 2^30 or more messages for one book (that
                                   book is left untouched)                        */

typedef struct {
  int32_t n_books;                       /* books in the context, >= 1             */
  const int32_t *capacity_host;          /* [n_books] orders per side, 1..4096      */
  int32_t l2_levels;                     /* L2 depth, 1..64 (the paper uses 10)     */
  int32_t device;                        /* HIP device ordinal                     */
  const int64_t *trade_log_records_host; /* [n_books] trade-log room per book, or  */
                                         /* NULL: trade_log_default for every book */
  int64_t trade_log_default;             /* records per book when the array is NULL */
  uint32_t flags;                        /* reserved, 0                            */
} lob_config;

/* Per-book counters since creation or the last lob_reset (lob_read_status). */
typedef struct {
  int64_t n_msgs;           /* messages handed to the book, of any type          */
  int64_t n_trades;         /* trades generated (including any dropped from log)  */
  int64_t limit_qty;        /* summed qty of limit messages with qty > 0          */
  int64_t market_qty;       /* summed qty of market messages with qty > 0         */
  int64_t traded_qty;       /* summed trade quantity                             */
  int64_t cancelled_qty;    /* quantity removed by cancel / delete               */
  int64_t market_discarded; /* unmatched remainder of market orders              */
  int64_t rejected_qty;     /* limit remainder rejected by a full side           */
  int64_t cancel_miss;      /* cancels / deletes that found no order             */
  int32_t flags;            /* LOB_BOOK_*                                        */
  int32_t n_live[2];        /* resting orders now: [0] asks, [1] bids            */
  int32_t pad;
  int64_t log_records;      /* trades waiting in the book's log                  */
} lob_book_status;

/* Execution plan (lob_set_plan).  Results never depend on the plan, only speed. */
typedef struct {
  int32_t lds_slots;       /* orders per side kept in LDS by lob_process_messages and
                              lob_step launches, 1..4096; a book with a larger
                              capacity keeps the orders past this many in HBM     */
  int32_t books_per_block; /* wavefronts (one book each) per workgroup, 1..16    */
  int32_t ragged_split;    /* lob_process_ragged: 0 = one launch with window
                              lds_slots; > 0 = books of capacity <= ragged_split
                              run in one launch with window ragged_split, the
                              others concurrently in a second launch with window
                              lds_slots_big                                     */
  int32_t lds_slots_big;   /* window of the second ragged launch, 1..4096        */
  int32_t ragged_order;    /* lob_process_ragged: 1 = longest stream first
                              (longest-processing-time list scheduling), 0 = as
                              listed                                            */
  int32_t books_per_block_big; /* books per workgroup of the second ragged launch */
  int32_t registers;       /* 1: while its messages run, each book keeps the first
                              128 orders of a side in registers -- the whole book
                              when the launch's capacities are <= 128, else with
                              the rest in LDS when that fits (larger books use the
                              LDS window); 0: always the LDS window             */
  int32_t layout;          /* 0: each side kept sorted in priority order (the
                              kernels above); 1: the paper's layout -- unsorted
                              fixed-size arrays, first free position for an add,
                              a search of the whole side per trade and per cancel
                              -- with the whole book in LDS (for comparison; same
                              results; capacity limited by LDS)                 */
  int32_t max_capacity;    /* lob_process_messages, lob_step and lob_exec_step: 0 =
                              size each launch for the context's largest capacity;
                              > 0 = the listed books' capacities are at most this,
                              and each launch takes the kernel form, window and
                              occupancy of that capacity (a listed book above it
                              is left untouched and flagged LOB_BOOK_BAD_LOAD).
                              lob_process_ragged and the server size each launch
                              from the capacities of the books it holds.        */
  int32_t tail_shallow;    /* 1: launches of books larger than 128 orders per side
                              (no agent fills, no per-message L2) take the code
                              laid out for sides the flow has drained below 64
                              orders (faster there, slower for books that stay
                              deep); 0 = laid out for deep books.  The ragged
                              autotuner tries both.                              */
} lob_plan;

typedef struct lob_ctx lob_ctx;

/* Create a context on cfg->device: n_books books, book i with room for
 * capacity_host[i] orders per side -- the fixed-size order arrays of Section 4
 * (eq. "features"), whose empty positions are all -1 -- every book empty, every
 * trade log empty, L2 snapshots of l2_levels levels (Section 5.1.1 uses 10).  All
 * device memory the context uses is allocated here (books, trade logs, staging).
 * Returns LOB_EINVAL (bad config), LOB_ENOMEM or LOB_EDEVICE; *out is NULL then. */
lob_status lob_create(const lob_config *cfg, lob_ctx **out);

/* Free the context and its device memory (waits for the device first). */
void lob_destroy(lob_ctx *ctx);

/* Text of the last error on this context (ctx == NULL: the last lob_create failure
 * on this thread).  Valid until the next call on the same context / thread. */
const char *lob_last_error(const lob_ctx *ctx);

/* Number of books, largest capacity and L2 depth of a context. */
lob_status lob_info(const lob_ctx *ctx, int32_t *n_books, int32_t *max_capacity,
                    int32_t *l2_levels);

/* Replace / read the execution plan.  Results never depend on the plan. */
lob_status lob_set_plan(lob_ctx *ctx, const lob_plan *plan);
lob_status lob_get_plan(const lob_ctx *ctx, lob_plan *plan);

/* Process message streams (Section 4.2, one message at a time per book).
 *   book_ids [n_books]    books to process (NULL: books 0..n_books-1)
 *   msgs     [..][8]      message records
 *   msg_offsets [n+1]     listed book i processes msgs[msg_offsets[i] ..
 *                         msg_offsets[i+1]) in order; offsets non-decreasing
 *   l2_mode, l2_out       LOB_L2_NONE (l2_out unused); LOB_L2_PER_MESSAGE:
 *                         l2_out[k] = snapshot after message k (k indexes msgs);
 *                         LOB_L2_FINAL: l2_out[i] = snapshot of listed book i at
 *                         the end; each snapshot is [2][levels][2]
 * Trades are appended to each book's trade log (lob_read_trades drains it).
 * The books' state stays on the device between calls. */
lob_status lob_process_messages(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books,
                                const int32_t *msgs, const int64_t *msg_offsets,
                                int32_t l2_mode, int32_t *l2_out, void *stream);

/* Ragged batches: books of uneven capacity and stream length in one call.  Same
 * results as lob_process_messages; the host also receives the stream bounds, so
 * the library can order the books longest stream first and split them into
 * capacity buckets that run concurrently (see lob_plan).  The workgroup dispatcher
 * hands each next book to the first free SIMD.
 *   book_ids_host [n_books]   host array of distinct book ids (NULL: 0..n-1),
 *                             checked on the host (LOB_EINVAL if out of range or
 *                             repeated)
 *   msg_offsets_host [n+1]    host array: listed book i processes
 *                             msgs[msg_offsets_host[i] .. msg_offsets_host[i+1])
 *   l2_mode, l2_out           as lob_process_messages (rows keep the listed order)
 * Waits for the host-to-device copy of the schedule of the previous ragged call
 * on this context before reusing its staging buffer. */
lob_status lob_process_ragged(lob_ctx *ctx, const int32_t *book_ids_host, int32_t n_books,
                              const int32_t *msgs, const int64_t *msg_offsets_host,
                              int32_t l2_mode, int32_t *l2_out, void *stream);

/* Autotuner for lob_process_ragged: runs the batch under candidate plans -- one
 * launch or two capacity buckets, the LDS engine or the paper's unsorted layout
 * (Section 4) in one launch, LDS window sizes (books larger than the window keep
 * their tail in HBM), books per workgroup -- times each candidate with HIP events
 * on `stream` as the slowest of three runs after one untimed run, installs the
 * fastest plan in the context and returns it with that time.  Every run starts
 * from empty books: the listed ids are checked (LOB_EINVAL if one is out of range,
 * before anything runs) and the listed books reset before each run and left reset
 * at the end (their previous state is lost).  At most max_trials candidates (>= 1),
 * four runs each (one when the untimed run already takes twice the best time so
 * far); a candidate that does not fit (LDS) is skipped and not counted.
 * Waits for the device (not graph-capturable). */
lob_status lob_autotune_ragged(lob_ctx *ctx, const int32_t *book_ids_host, int32_t n_books,
                               const int32_t *msgs, const int64_t *msg_offsets_host,
                               int32_t max_trials, lob_plan *best, float *best_ms, void *stream);

/* One environment step per listed book (Section 5.1.3): the W data messages of
 * window[i] (zero padding skipped), then the A agent messages of actions[i]
 * (type 0 = no order), then the book's L2 snapshot into l2_out[i] and the trades
 * of this step in which either side carries trader id agent_tid into
 * agent_fills[i][0..F) (trade records, in order); agent_fill_counts[i] receives
 * their number (more than F: the rest are dropped and flagged).  The step's trades
 * are not appended to the trade log.  Allocates nothing and never waits for the
 * device, so a sequence of steps can be captured in a HIP graph.
 *   window [n][W][8], actions [n][A][8] (A may be 0, actions NULL),
 *   l2_out [n][2][levels][2], agent_fills [n][F][6] (F may be 0),
 *   agent_fill_counts [n] (may be NULL when F == 0). */
lob_status lob_step(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books,
                    const int32_t *window, int32_t W, const int32_t *actions, int32_t A,
                    int32_t agent_tid, int32_t *l2_out, int32_t *agent_fills, int32_t F,
                    int32_t *agent_fill_counts, void *stream);

/* Current L2 snapshot of each listed book into l2_out [n][2][levels][2]: the
 * ten-level (or l2_levels) book state the environment of Section 5.1.1 observes,
 * in the L2 layout above. */
lob_status lob_read_l2(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, int32_t *l2_out,
                       void *stream);

/* Drain trade logs.  counts[i] = records waiting in listed book i's log;
 * offsets[0..n] = exclusive prefix sum of counts (offsets[n] = total).  Book i's
 * records are copied, oldest first, to out[offsets[i] ..) as 6-int32 records and
 * its log is emptied -- but only if offsets[i+1] <= max_records; a book that does
 * not fit is left as it is (compare offsets[n] with max_records and call again
 * with more room).  counts and offsets are device int64 arrays. */
lob_status lob_read_trades(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, int32_t *out,
                           int64_t max_records, int64_t *counts, int64_t *offsets,
                           void *stream);

/* Per-book counters and flags into out[n] (device memory). */
lob_status lob_read_status(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books,
                           lob_book_status *out, void *stream);

/* Checkpoint / restore: a book dump [n][2][dump_cap][6] per listed book.
 * lob_read_book writes each side in priority order (rows past the live orders, or
 * past dump_cap, are -1 / cut off).  lob_write_book replaces each listed book's
 * orders by the dump's rows, taken in the given order up to the first row with
 * Q <= 0 or the book's capacity; the rows must be in priority order (as
 * lob_read_book writes them: prices best first, equal prices by time), else the
 * book is flagged LOB_BOOK_BAD_LOAD.  The book's latest time becomes at least the
 * newest written order's, so that a later message stamped before it counts as
 * time going backwards.  Counters and trade logs are not touched. */
lob_status lob_read_book(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, int32_t *out,
                         int32_t dump_cap, void *stream);
lob_status lob_write_book(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books,
                          const int32_t *in, int32_t dump_cap, void *stream);

/* Empty the listed books, their trade logs and their counters. */
lob_status lob_reset(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, void *stream);

/* Start each listed book from an L2 snapshot, as JAX-LOB starts an episode window
 * (Section 5.1.1).  l2 is device [n_books][2][levels][2] in lob_read_l2's layout:
 * side 0 asks best first (ascending prices), side 1 bids best first (descending),
 * entries (price, qty), qty <= 0 = missing level; levels in 1..LOB_MAX_LEVELS.
 * Each book is emptied together with its counters and trade log, then every
 * present level becomes ONE order holding the level's quantity (the snapshot does
 * not tell the orders of a level apart): order ids -9000, -9001, ... handed out
 * level by level with the ask before the bid (the column order of a LOBSTER
 * order-book row), trader id init_tid, time times[i] = (Ts, Tns) (device
 * [n_books][2], NULL = (0, 0)), which also becomes the book's latest time (a later
 * message stamped before it is flagged like any time going backwards).  Such
 * orders are what the cancel rule for initial
 * orders (id <= -9000, matched by price) acts on.  A snapshot that is not a book
 * -- prices not strictly ordered on a side, best bid >= best ask, or more levels
 * on a side than the capacity -- leaves the book empty with LOB_BOOK_BAD_LOAD. */
lob_status lob_seed_l2(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, const int32_t *l2, int32_t levels,
                       const int32_t *times, int32_t init_tid, void *stream);

/* Diagnostic: run the wavefront primitives the matcher is built on on one
 * wavefront and write 576 int32 results to out (device), with x = 3*lane + 1:
 * [0,64) inclusive prefix sums of (lane % 7 + 1); [64,128) number of lanes <=
 * lane with lane % 3 == 0; [128,192) number of lanes below lane; [192,256) x of
 * lane-1 (lane 0: -5); [256,320) x of lane+1 (lane 63: -7); [320,384) x of lane
 * (lane+5) % 64; [384,448) x of lane-1 (lane 0: 0); [448,512) x of lane+1
 * (lane 63: 0); [512,576) x with lane 17 replaced by -9. */
lob_status lob_selftest(int32_t device, int32_t *out, void *stream);

/* ---------------------------------------------------------------- execution environment */

/* Per-book state of an execution task (Section 5.2), device memory, one per listed
 * book; lob_exec_step reads and updates it.  The caller fills it at the episode
 * start (exec_qty = revenue = done = flags = 0). */
typedef struct {
  int32_t task_side;  /* +1: buy task_qty shares; -1: sell them                      */
  int32_t task_qty;   /* Q_task                                                      */
  int32_t exec_qty;   /* Q_exec: agent quantity executed so far, at most Q_task (upd.) */
  int32_t done;       /* 1 once Q_exec = Q_task or the episode time is over (upd.)   */
  int64_t revenue;    /* sum of P_j * Q_j over the counted agent fills (updated)     */
  int32_t p_init;     /* P_init: mid price at the episode start                      */
  int32_t start_s;    /* episode start time (Ts, Tns)                                */
  int32_t start_ns;
  int32_t end_s;      /* episode end (s); from end_s - 60 on, the remaining quantity
                         is submitted as one market order instead of the action     */
  int32_t next_oid;   /* order id of the agent's next order (updated)                */
  int32_t flags;      /* LOB_EXEC_* (updated)                                        */
} lob_exec_state;     /* 48 bytes */

#define LOB_EXEC_TRADES_MISSING 1 /* the trade log had no room for some of a step's
                                     trades: that step's VWAP misses them          */
#define LOB_EXEC_FILLS_MISSING 2  /* a step had more agent fills than F and the
                                     first F did not finish the task: Q_exec, the
                                     revenue and the reward miss the others       */

typedef struct {
  int32_t tick;          /* tick size in price units                                 */
  int32_t passive_ticks; /* n of the passive price                                   */
  int32_t agent_tid;     /* trader id carried by the agent's orders                  */
  int32_t keep_trades;   /* 0: the step's trades leave the trade log once the reward
                            is computed; 1: they stay for lob_read_trades           */
  double lambda;         /* weight of the drift term of the reward                   */
} lob_exec_params;

/* One step of the execution environment of Section 5.2 per listed book, three
 * kernels on `stream`, allocating nothing:
 *  1. the action -- sizes action_qty[i][0..4) at the far-touch, mid, near-touch and
 *     passive prices of the book as it stands (buy task: ask, floor((ask+bid)/2),
 *     bid, bid - passive_ticks*tick; sell task: bid, mid, ask, ask + passive_ticks*
 *     tick) -- becomes up to four limit orders (size <= 0, or a reference price
 *     missing or <= 0: no order), ids state.next_oid, next_oid+1, ..., trader id
 *     agent_tid, time of the step's last data message.  From end_s - 60 on, one
 *     market order for Q_task - Q_exec replaces them; a done task sends nothing.
 *  2. the W data messages of window[i] then those orders run through the matcher
 *     (lob_step's semantics; the trades are logged for step 3).
 *  3. obs[i] (6W + 8 int32): best bid prices after each data message [W], best ask
 *     prices [W], mid prices floor((ask+bid)/2) [W], passive prices [W], spreads
 *     ask - bid [W], level-1 imbalances Q_ask - Q_bid [W] (a missing best price
 *     reads -1; mid, passive and spread read -1 when a price they need is
 *     missing; a missing side's quantity is 0), then the current time (Ts, Tns) =
 *     the step's last data message, the elapsed time (Ts, Tns) since the episode
 *     start, P_init, the drift P_mid - P_init (P_mid of the last data message; 0
 *     if missing), Q_task and Q_exec.  reward[i] (float64) =
 *       sum_j Q_j (P_j - P_VWAP) + lambda * sum_j Q_j (P_VWAP - P_init),
 *     P_VWAP = sum_i Q_i P_i / sum_i Q_i over all trades of the step, j over the
 *     agent's fills of the step with Q_j capped so that Q_exec never exceeds
 *     Q_task (0 when the step made no trade); computed from exact int64 sums in
 *     that order with no fused operations.  The agent's fills go to
 *     agent_fills[i] / agent_fill_counts[i] as in lob_step; state is updated.
 * W in 1..256; the trade log of a book needs room for the step's trades (2 per
 * message at most), else LOB_EXEC_TRADES_MISSING.  A step makes at most
 * 2 * capacity + W + 4 agent fills (each fill empties its standing order or its
 * aggressor): with F at least that, Q_exec, the revenue and the reward count every
 * fill; with a smaller F they are still exact when the first F fills finish the
 * task, else the step sets LOB_EXEC_FILLS_MISSING.  window [n][W][8], action_qty
 * [n][4], state [n], obs [n][6W+8], reward [n], agent_fills [n][F][6] with F >= 1,
 * agent_fill_counts [n]; all device memory, obs 4-byte aligned. */
lob_status lob_exec_step(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, const int32_t *window,
                         int32_t W, const int32_t *action_qty, const lob_exec_params *params,
                         lob_exec_state *state, int32_t *obs, double *reward, int32_t *agent_fills, int32_t F,
                         int32_t *agent_fill_counts, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): lob_exec_step with the same arguments, results
 * and stream semantics, whose agent-order staging and step bookkeeping live in a
 * static array of the library (2.25 MiB per GPU, held until the process ends)
 * instead of the context's buffers.  It calls no allocating routine.  At most
 * LOB_NOALLOC_MAX_BOOKS books per call (LOB_ECAP beyond).  Every call on one GPU
 * uses that GPU's one array: calls that overlap on the device (other streams,
 * other contexts, other host threads) race and must be serialised by the caller. */
#define LOB_NOALLOC_MAX_BOOKS 16384
lob_status lob_exec_step_noalloc(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, const int32_t *window,
                                 int32_t W, const int32_t *action_qty, const lob_exec_params *params,
                                 lob_exec_state *state, int32_t *obs, double *reward, int32_t *agent_fills,
                                 int32_t F, int32_t *agent_fill_counts, void *stream);

/* ---------------------------------------------------------------- replay windows */

/* Windowed replay data (Section 5.1.1, data loading).  Host memory only, no GPU
 * work.  One book's stream msgs_host[n_msgs][8], times not decreasing, is cut into
 * n_windows consecutive windows of window_s seconds, window k holding the
 * messages with start_s + k*window_s <= Ts < start_s + (k+1)*window_s (messages
 * before start_s or past the last window are in none), and each window into steps
 * of msgs_per_step messages.  out_host [n_windows][max_steps][msgs_per_step][8]
 * (or NULL: only count) receives each window's messages in order, the rest of its
 * last step and the steps after it all-zero (type 0: the step form never
 * processes them); steps_host[k] = steps of window k that hold messages (the
 * episode of that window ends after them); first_host[k] = index of window k's
 * first message, first_host[n_windows] = one past the last window's messages.
 * Returns LOB_ECAP when a window needs more than max_steps steps (it is cut off
 * at max_steps and steps_host says max_steps; call with out_host = NULL to size),
 * LOB_EINVAL for bad sizes or a time that goes back across a window boundary. */
lob_status lob_windows(const int32_t *msgs_host, int64_t n_msgs, int32_t start_s, int32_t window_s,
                       int32_t msgs_per_step, int32_t max_steps, int32_t n_windows, int32_t *out_host,
                       int32_t *steps_host, int64_t *first_host);

/* ---------------------------------------------------------------- serving */

/* A request loop over the books of one context: requests arrive one by one, each
 * for one book -- a replay request (messages; returns the trades they make) or a
 * step request (messages, then up to 4 agent orders; returns the book's L2 and
 * the step's agent fills).  The server keeps at most one request per book on the
 * device, so every book sees its requests in arrival order; it gathers whatever
 * has arrived into a batch whenever a batch slot (stream) is free and the batch
 * fits the slot's share of the HBM staging budget, so batches run while new ones
 * are formed.  Book state stays resident in the context between requests. */
#define LOB_REQ_REPLAY 0
#define LOB_REQ_STEP 1

typedef struct {
  int32_t n_slots;        /* batches in flight at once, each on its own stream, 1..16 */
  int64_t hbm_budget;     /* bytes of device staging shared by the slots (inputs,
                             outputs, trades room); a request waits until it fits */
  int32_t max_batch;      /* requests per batch, >= 1                              */
  int32_t max_request_msgs; /* largest request accepted (messages)                 */
  int32_t fill_cap;       /* agent fills kept per step request on the device        */
  int32_t agent_tid;      /* trader id that marks the agent's orders                */
} lob_server_config;

typedef struct {
  int64_t tag;                 /* caller's id, echoed in the completion             */
  int32_t book;                /* book id in the context                            */
  int32_t kind;                /* LOB_REQ_REPLAY or LOB_REQ_STEP                    */
  const int32_t *msgs_host;    /* [n_msgs][8] message records                       */
  int32_t n_msgs;              /* 0..max_request_msgs                               */
  int32_t n_actions;           /* step: agent messages in actions_host, 0..4        */
  const int32_t *actions_host; /* [n_actions][8]                                    */
  int32_t *trades_host;        /* replay: room for trades_room trade records        */
  int32_t trades_room;
  int32_t *l2_host;            /* step: [2][levels][2]                              */
  int32_t *fills_host;         /* step: room for fills_room trade records           */
  int32_t fills_room;
} lob_request;
/* All host buffers of a request must stay valid until its completion is returned. */

typedef struct {
  int64_t tag;
  int32_t status;       /* LOB_OK, or LOB_ECAP when the trades / fills did not all fit
                           (the caller's room or fill_cap); n_out is still exact      */
  int32_t n_out;        /* trades (replay) or agent fills (step) the request made    */
  int64_t arrival_ns;   /* server clock (lob_server_now) at arrival                  */
  int64_t launch_ns;    /* when its batch was handed to the GPU                      */
  int64_t complete_ns;  /* when its results were in the caller's host buffers        */
} lob_completion;

typedef struct lob_server lob_server;

/* Allocates every staging buffer the server uses (device and pinned host). */
lob_status lob_server_create(lob_ctx *ctx, const lob_server_config *cfg, lob_server **out);
/* Waits for the batches in flight, then frees the server (not the context). */
void lob_server_destroy(lob_server *srv);
/* Nanoseconds on the server's clock (steady, since creation). */
int64_t lob_server_now(const lob_server *srv);
/* Queue a request that arrived at arrival_ns (server clock); no GPU work. */
lob_status lob_server_submit(lob_server *srv, const lob_request *req, int64_t arrival_ns);
/* Advance: retire finished batches (results copied to the requests' buffers),
 * launch new batches from the queue; up to max_out completions into out. */
lob_status lob_server_poll(lob_server *srv, lob_completion *out, int32_t max_out, int32_t *n_out);
/* Open-loop driver: request k arrives arrival_ns[k] after the call starts
 * (non-decreasing); submits each at its time and polls until all n have
 * completed; completions go to out[0..n) in completion order. */
lob_status lob_server_run(lob_server *srv, const lob_request *reqs, const int64_t *arrival_ns, int64_t n,
                          lob_completion *out);

#ifdef __cplusplus
}
#endif
#endif
