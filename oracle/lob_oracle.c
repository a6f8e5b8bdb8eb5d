/*
 * lob_oracle.c -- reference oracle: the plain sequential matching engine of
 * JAX-LOB (Frey et al. 2023), Section 4, for use by tests only.
 *
 * TEST INFRASTRUCTURE ONLY (see lob_oracle.h).  Deliberately slow and literal:
 * unsorted fixed-size arrays, a full scan for every best-order search, and the
 * clean-up pass over both sides after every basic operation.
 *
 * Readings of the paper taken here (each also applies at the marked place):
 *   R1  The best bid is the HIGHEST bid price; eq. "best_price" prints min for
 *       both sides, which for bids contradicts price-time priority (Section 4.1).
 *   R2  Among equal prices the earliest (Ts, Tns) wins; orders with equal times
 *       are ranked by arrival order (the paper is silent on equal times).
 *   R3  The price overlap test of the matching loop is inclusive (Section 4.1).
 *   R4  A limit remainder that finds its side full is rejected and counted; the
 *       paper only asks that N be large enough never to saturate (Section 4).
 *   R5  Cancel and delete search the message's side for the message's OID; if
 *       several live orders carry it, the best-priority one is used.  If none
 *       does, the initial-order rule of Section 5.1.1 applies with the bound read
 *       as OID <= -9000 (the text says ids start at -9000 but tests < -9000);
 *       the best-priority match wins.  A cancel that finds nothing is a no-op and
 *       is counted as a miss.
 *   R6  A cancel or delete with Q <= 0 is a no-op (a negative Q would add shares);
 *       delete subtracts its Q like cancel does ("treated identically", 4.2).
 *   R7  Message types outside 1..4 are no-ops: the zero-padded steps of
 *       Section 5.1.1 are never processed.  A side other than +1 / -1 is a no-op.
 *   R8  A limit or market message with Q <= 0 trades nothing and rests nothing,
 *       which is what add-then-clean-up gives (Table 2 uses Q_a = 0).
 *   R14 Book initialisation from an L2 snapshot (Section 5.1.1): one order per
 *       level with the level's summed quantity; the ids -9000, -9001, ... are
 *       handed out level by level, ask before bid, the column order of a LOBSTER
 *       order-book row.  The paper leaves trader id and time of these orders open:
 *       both are arguments.  A snapshot that is not a valid book is refused.  The
 *       initial orders' time counts as the book's latest time, so a later message
 *       stamped before it is flagged like any other time going backwards (R2).
 *   R19 Quantities are int32 (Section 4.2).  Matching, cancels and the counters
 *       stay exact for every int32 quantity (the counters are int64).  An L2
 *       level's summed quantity, which can pass INT32_MAX, is summed exactly and
 *       reported as min(sum, INT32_MAX): the L2 record is int32 and the paper does
 *       not define a level beyond it.
 */
#include "lob_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* order fields, eq. "features" */
enum { P = 0, Q = 1, OID = 2, TID = 3, TS = 4, TNS = 5 };
/* message fields as stored */
enum { M_T = 0, M_S = 1, M_P = 2, M_Q = 3, M_OID = 4, M_TID = 5, M_TS = 6, M_TNS = 7 };

typedef struct {
  int32_t f[ORC_ORDER_FIELDS];
  int64_t arrival; /* R2: rank among equal times; -1 when empty */
} order_t;

struct orc_book {
  int32_t N;
  order_t *A; /* asks, Section 4: A = [a_1 .. a_N] */
  order_t *B; /* bids, Section 4: B = [b_1 .. b_N] */
  int64_t next_arrival;
  int32_t last_ts, last_tns;
  int32_t seen_time;
  orc_stats st;
};

static void set_empty(order_t *o) {
  for (int k = 0; k < ORC_ORDER_FIELDS; ++k) o->f[k] = -1;
  o->arrival = -1;
}

/* Section 4: an empty position has all six features equal to -1. */
static int is_empty(const order_t *o) {
  for (int k = 0; k < ORC_ORDER_FIELDS; ++k)
    if (o->f[k] != -1) return 0;
  return 1;
}

orc_book *orc_new(int32_t N) {
  if (N < 1) return NULL;
  orc_book *b = (orc_book *)calloc(1, sizeof(orc_book));
  if (!b) return NULL;
  b->N = N;
  b->A = (order_t *)malloc(sizeof(order_t) * (size_t)N);
  b->B = (order_t *)malloc(sizeof(order_t) * (size_t)N);
  if (!b->A || !b->B) {
    orc_free(b);
    return NULL;
  }
  for (int32_t i = 0; i < N; ++i) {
    set_empty(&b->A[i]);
    set_empty(&b->B[i]);
  }
  return b;
}

void orc_free(orc_book *b) {
  if (!b) return;
  free(b->A);
  free(b->B);
  free(b);
}

int32_t orc_capacity(const orc_book *b) { return b->N; }
void orc_get_stats(const orc_book *b, orc_stats *out) { *out = b->st; }

/* Section 4.1, last paragraph of the list: after every operation both sides are
 * checked for orders with Q <= 0, which are set to -1. */
static void cleanup(orc_book *b) {
  for (int32_t i = 0; i < b->N; ++i) {
    if (b->A[i].f[Q] <= 0) set_empty(&b->A[i]);
    if (b->B[i].f[Q] <= 0) set_empty(&b->B[i]);
  }
}

/* Is x ahead of y in price-time priority on a side?  (eq. best_price, R1, R2) */
static int ahead(const order_t *x, const order_t *y, int is_bid_side) {
  if (x->f[P] != y->f[P]) return is_bid_side ? x->f[P] > y->f[P] : x->f[P] < y->f[P];
  if (x->f[TS] != y->f[TS]) return x->f[TS] < y->f[TS];
  if (x->f[TNS] != y->f[TNS]) return x->f[TNS] < y->f[TNS];
  return x->arrival < y->arrival;
}

/* Best(o_s): index of the best order on a side, -1 if the side is empty. */
static int32_t best(const order_t *side, int32_t N, int is_bid_side) {
  int32_t b = -1;
  for (int32_t i = 0; i < N; ++i) {
    if (is_empty(&side[i])) continue;
    if (b < 0 || ahead(&side[i], &side[b], is_bid_side)) b = i;
  }
  return b;
}

typedef struct {
  int32_t *buf;
  int32_t room;
  int32_t n;
} sink_t;

static void log_trade(sink_t *s, const int32_t *t) {
  if (s->n < s->room) memcpy(s->buf + (size_t)s->n * ORC_TRADE_FIELDS, t, sizeof(int32_t) * ORC_TRADE_FIELDS);
  s->n++;
}

/* Matching (Section 4.1, item 3 and the while-loop that follows it).  The
 * aggressive order o_a with limit price P_a and quantity Q_a is matched against
 * the best standing order o_s on the opposite side while that side is non-empty,
 * Q_a > 0 and the prices overlap (inclusive, R3).  Returns the final Q_a. */
static int32_t match(orc_book *b, int aggressor_buys, int32_t P_a, int32_t Q_a, const int32_t *m,
                     sink_t *sink) {
  order_t *opp = aggressor_buys ? b->A : b->B;
  for (;;) {
    if (!(Q_a > 0)) break;
    int32_t s = best(opp, b->N, !aggressor_buys);
    if (s < 0) break; /* the opposite side is empty */
    order_t *o_s = &opp[s];
    int32_t P_s = o_s->f[P], Q_s = o_s->f[Q];
    int overlap = aggressor_buys ? (P_a >= P_s) : (P_a <= P_s);
    if (!overlap) break;
    /* Q_s' = max(0, Q_s - Q_a),  Q_a' = Q_a - Q_s */
    int32_t Q_s_new = Q_s - Q_a > 0 ? Q_s - Q_a : 0;
    int32_t Q_a_new = Q_a - Q_s;
    /* t_j: P_j = P_s, Q_j = Q_s - Q_s', both order ids, Ts_j, Tns_j = Ts_a, Tns_a */
    int32_t t[ORC_TRADE_FIELDS];
    t[0] = P_s;
    t[1] = Q_s - Q_s_new;
    t[2] = o_s->f[OID];
    t[3] = m[M_OID];
    t[4] = m[M_TS];
    t[5] = m[M_TNS];
    t[6] = o_s->f[TID];
    t[7] = m[M_TID];
    log_trade(sink, t);
    b->st.n_trades++;
    b->st.traded_qty += t[1];
    o_s->f[Q] = Q_s_new;
    Q_a = Q_a_new;
    cleanup(b);
  }
  return Q_a;
}

/* Addition (Section 4.1, item 1): write the order into an empty position. */
static void add(orc_book *b, int bid_side, const int32_t *m, int32_t qty) {
  order_t *own = bid_side ? b->B : b->A;
  int32_t slot = -1;
  for (int32_t i = 0; i < b->N; ++i)
    if (is_empty(&own[i])) {
      slot = i;
      break;
    }
  if (slot < 0) { /* R4 */
    b->st.rejected_qty += qty;
    b->st.flags |= ORC_FLAG_SIDE_FULL;
    return;
  }
  order_t *o = &own[slot];
  o->f[P] = m[M_P];
  o->f[Q] = qty;
  o->f[OID] = m[M_OID];
  o->f[TID] = m[M_TID];
  o->f[TS] = m[M_TS];
  o->f[TNS] = m[M_TNS];
  o->arrival = b->next_arrival++;
  cleanup(b);
}

/* Cancellation (Section 4.1, item 2; Section 5.1.1 for initial orders; R5, R6). */
static void cancel(orc_book *b, int bid_side, const int32_t *m) {
  if (m[M_Q] <= 0) return; /* R6 */
  order_t *own = bid_side ? b->B : b->A;
  int32_t k = -1;
  for (int32_t i = 0; i < b->N; ++i) {
    if (is_empty(&own[i]) || own[i].f[OID] != m[M_OID]) continue;
    if (k < 0 || ahead(&own[i], &own[k], bid_side)) k = i;
  }
  if (k < 0) {
    for (int32_t i = 0; i < b->N; ++i) {
      if (is_empty(&own[i]) || !(own[i].f[OID] <= -9000 && own[i].f[P] == m[M_P])) continue;
      if (k < 0 || ahead(&own[i], &own[k], bid_side)) k = i;
    }
  }
  if (k < 0) {
    b->st.cancel_miss++;
    return;
  }
  b->st.cancelled_qty += m[M_Q] < own[k].f[Q] ? m[M_Q] : own[k].f[Q];
  own[k].f[Q] -= m[M_Q];
  cleanup(b);
}

int32_t orc_process(orc_book *b, const int32_t *m, int32_t *trades, int32_t max_trades) {
  sink_t sink = {trades, trades ? max_trades : 0, 0};
  int32_t T = m[M_T], S = m[M_S];
  b->st.n_msgs++;
  if (T < 1 || T > 4) return 0;   /* R7: padding */
  if (S != 1 && S != -1) return 0; /* R7 */
  if (b->seen_time && (m[M_TS] < b->last_ts || (m[M_TS] == b->last_ts && m[M_TNS] < b->last_tns)))
    b->st.flags |= ORC_FLAG_TIME_ORDER;
  b->seen_time = 1;
  b->last_ts = m[M_TS];
  b->last_tns = m[M_TNS];
  int buys = (S == 1);
  if (T == 1) {
    /* Section 4.2, item 1: match first, then add the remainder as one new order. */
    if (m[M_Q] > 0) b->st.limit_qty += m[M_Q];
    int32_t rem = match(b, buys, m[M_P], m[M_Q], m, &sink);
    if (rem > 0) add(b, buys, m, rem); /* R8 */
  } else if (T == 4) {
    /* Section 4.2, item 3: price 0 for a sell, max_int for a buy; the unmatched
     * quantity is disregarded.  The message's price field is ignored. */
    if (m[M_Q] > 0) b->st.market_qty += m[M_Q];
    int32_t P_m = buys ? INT32_MAX : 0;
    int32_t rem = match(b, buys, P_m, m[M_Q], m, &sink);
    if (rem > 0) b->st.market_discarded += rem;
  } else {
    /* Section 4.2, item 2: cancel (T=2) and delete (T=3) are the same operation. */
    cancel(b, buys, m);
  }
  return sink.n;
}

/* L2 (Section 5.1.1 uses ten levels): per side, the distinct prices best first,
 * each with the summed quantity of its orders; missing levels are (-1, 0). */
void orc_l2(const orc_book *b, int32_t levels, int32_t *out) {
  for (int sd = 0; sd < 2; ++sd) {
    const order_t *side = sd == 0 ? b->A : b->B;
    int is_bid = (sd == 1);
    int have_prev = 0;
    int32_t prev = 0;
    for (int32_t l = 0; l < levels; ++l) {
      /* the best price strictly behind the previous level */
      int found = 0;
      int32_t px = 0;
      for (int32_t i = 0; i < b->N; ++i) {
        if (is_empty(&side[i])) continue;
        int32_t p = side[i].f[P];
        if (have_prev && !(is_bid ? p < prev : p > prev)) continue;
        if (!found || (is_bid ? p > px : p < px)) {
          px = p;
          found = 1;
        }
      }
      int32_t *o = out + ((size_t)sd * levels + l) * 2;
      if (!found) {
        o[0] = -1;
        o[1] = 0;
        continue;
      }
      int64_t qsum = 0; /* R19 */
      for (int32_t i = 0; i < b->N; ++i)
        if (!is_empty(&side[i]) && side[i].f[P] == px) qsum += side[i].f[Q];
      o[0] = px;
      o[1] = qsum > INT32_MAX ? INT32_MAX : (int32_t)qsum;
      prev = px;
      have_prev = 1;
    }
  }
}

int32_t orc_dump(const orc_book *b, int32_t side, int32_t *out) {
  const order_t *s = side == 1 ? b->B : b->A;
  int is_bid = (side == 1);
  for (int32_t i = 0; i < b->N * ORC_ORDER_FIELDS; ++i) out[i] = -1;
  /* selection by repeated best-of-the-rest: plain and obviously ordered */
  char *taken = (char *)calloc((size_t)b->N, 1);
  if (!taken) return -1;
  int32_t n = 0;
  for (;;) {
    int32_t k = -1;
    for (int32_t i = 0; i < b->N; ++i) {
      if (taken[i] || is_empty(&s[i])) continue;
      if (k < 0 || ahead(&s[i], &s[k], is_bid)) k = i;
    }
    if (k < 0) break;
    taken[k] = 1;
    memcpy(out + (size_t)n * ORC_ORDER_FIELDS, s[k].f, sizeof(int32_t) * ORC_ORDER_FIELDS);
    n++;
  }
  free(taken);
  return n;
}

/* Section 5.1.1: the book at the start of a window comes from its L2 snapshot (R14). */
int32_t orc_seed_l2(orc_book *b, const int32_t *l2, int32_t levels, int32_t tid, int32_t ts, int32_t tns) {
  for (int32_t i = 0; i < b->N; ++i) {
    set_empty(&b->A[i]);
    set_empty(&b->B[i]);
  }
  memset(&b->st, 0, sizeof(b->st));
  b->next_arrival = 0;
  /* R14: the initial orders' time is the book's latest time */
  b->seen_time = 1;
  b->last_ts = ts;
  b->last_tns = tns;
  /* is it a book?  strictly ordered prices per side, room for every level, not crossed */
  int ok = 1;
  int32_t best_px[2] = {0, 0};
  for (int sd = 0; sd < 2; ++sd) {
    int32_t count = 0, prev = 0;
    for (int32_t l = 0; l < levels; ++l) {
      const int32_t *e = l2 + ((size_t)sd * levels + l) * 2;
      if (e[1] <= 0) continue;
      if (count > 0 && (sd == 0 ? e[0] <= prev : e[0] >= prev)) ok = 0;
      if (count == 0) best_px[sd] = e[0];
      prev = e[0];
      count++;
    }
    if (count > b->N) ok = 0;
    if (count == 0) best_px[sd] = sd == 0 ? INT32_MAX : INT32_MIN;
  }
  if (best_px[1] >= best_px[0]) ok = 0;
  if (!ok) {
    b->st.flags |= ORC_FLAG_BAD_LOAD;
    return -1;
  }
  int32_t oid = -9000, placed = 0;
  for (int32_t l = 0; l < levels; ++l) {
    for (int sd = 0; sd < 2; ++sd) {
      const int32_t *e = l2 + ((size_t)sd * levels + l) * 2;
      if (e[1] <= 0) continue;
      order_t *own = sd == 1 ? b->B : b->A;
      int32_t slot = 0;
      while (!is_empty(&own[slot])) slot++; /* room was checked above */
      own[slot].f[P] = e[0];
      own[slot].f[Q] = e[1];
      own[slot].f[OID] = oid--;
      own[slot].f[TID] = tid;
      own[slot].f[TS] = ts;
      own[slot].f[TNS] = tns;
      own[slot].arrival = b->next_arrival++;
      placed++;
    }
  }
  return placed;
}

/* ---------------------------------------------------------------- batch runner */

typedef struct {
  int32_t n_books;
  const int32_t *caps;
  const int32_t *msgs;
  const int64_t *offs;
  int32_t l2_mode, levels;
  int32_t *l2_out;
  int32_t *trades;
  const int64_t *trade_offs;
  int64_t *trade_msg;
  int64_t *trade_counts;
  orc_stats *stats;
  int32_t *dumps;
  int32_t dump_cap;
  int32_t next; /* next book to take, guarded by mu */
  pthread_mutex_t mu;
  int32_t failed;
} job_t;

static int run_book(job_t *j, int32_t i) {
  orc_book *b = orc_new(j->caps[i]);
  if (!b) return -1;
  int32_t N = j->caps[i];
  int32_t *scratch = (int32_t *)malloc(sizeof(int32_t) * ORC_TRADE_FIELDS * (size_t)N);
  if (!scratch) {
    orc_free(b);
    return -1;
  }
  int64_t stored = 0, room = 0;
  int32_t *tbase = NULL;
  if (j->trades && j->trade_offs) {
    room = j->trade_offs[i + 1] - j->trade_offs[i];
    tbase = j->trades + (size_t)j->trade_offs[i] * ORC_TRADE_FIELDS;
  }
  int64_t generated = 0;
  for (int64_t k = j->offs[i]; k < j->offs[i + 1]; ++k) {
    int32_t nt = orc_process(b, j->msgs + (size_t)k * ORC_MSG_FIELDS, scratch, N);
    for (int32_t t = 0; t < nt; ++t) {
      if (tbase && stored < room) {
        memcpy(tbase + (size_t)stored * ORC_TRADE_FIELDS, scratch + (size_t)t * ORC_TRADE_FIELDS,
               sizeof(int32_t) * ORC_TRADE_FIELDS);
        if (j->trade_msg) j->trade_msg[j->trade_offs[i] + stored] = k;
        stored++;
      } else if (tbase) {
        b->st.flags |= ORC_FLAG_TRADE_FULL;
      }
    }
    generated += nt;
    if (j->l2_mode == ORC_L2_PER_MESSAGE)
      orc_l2(b, j->levels, j->l2_out + (size_t)k * 2 * j->levels * 2);
  }
  if (j->l2_mode == ORC_L2_FINAL) orc_l2(b, j->levels, j->l2_out + (size_t)i * 2 * j->levels * 2);
  if (j->trade_counts) j->trade_counts[i] = generated;
  if (j->stats) j->stats[i] = b->st;
  if (j->dumps) {
    int32_t *d = j->dumps + (size_t)i * 2 * j->dump_cap * ORC_ORDER_FIELDS;
    for (int32_t r = 0; r < 2 * j->dump_cap * ORC_ORDER_FIELDS; ++r) d[r] = -1;
    int32_t *full = (int32_t *)malloc(sizeof(int32_t) * ORC_ORDER_FIELDS * (size_t)N);
    if (!full) {
      free(scratch);
      orc_free(b);
      return -1;
    }
    for (int sd = 0; sd < 2; ++sd) {
      int32_t n = orc_dump(b, sd == 0 ? -1 : 1, full);
      int32_t keep = n < j->dump_cap ? n : j->dump_cap;
      memcpy(d + (size_t)sd * j->dump_cap * ORC_ORDER_FIELDS, full, sizeof(int32_t) * ORC_ORDER_FIELDS * (size_t)keep);
    }
    free(full);
  }
  free(scratch);
  orc_free(b);
  return 0;
}

static void *worker(void *arg) {
  job_t *j = (job_t *)arg;
  for (;;) {
    pthread_mutex_lock(&j->mu);
    int32_t i = j->next++;
    pthread_mutex_unlock(&j->mu);
    if (i >= j->n_books) break;
    if (run_book(j, i) != 0) {
      pthread_mutex_lock(&j->mu);
      j->failed = 1;
      pthread_mutex_unlock(&j->mu);
    }
  }
  return NULL;
}

int32_t orc_run(int32_t n_books, const int32_t *caps, const int32_t *msgs, const int64_t *offs,
                int32_t l2_mode, int32_t levels, int32_t *l2_out, int32_t *trades,
                const int64_t *trade_offs, int64_t *trade_msg, int64_t *trade_counts,
                orc_stats *stats, int32_t *dumps, int32_t dump_cap, int32_t n_threads) {
  if (n_books < 0 || !caps || !offs || (n_books > 0 && !msgs)) return -1;
  if (l2_mode != ORC_L2_NONE && (!l2_out || levels < 1)) return -1;
  if (dumps && dump_cap < 1) return -1;
  for (int32_t i = 0; i < n_books; ++i)
    if (caps[i] < 1 || offs[i + 1] < offs[i]) return -1;
  job_t j;
  memset(&j, 0, sizeof(j));
  j.n_books = n_books;
  j.caps = caps;
  j.msgs = msgs;
  j.offs = offs;
  j.l2_mode = l2_mode;
  j.levels = levels;
  j.l2_out = l2_out;
  j.trades = trades;
  j.trade_offs = trade_offs;
  j.trade_msg = trade_msg;
  j.trade_counts = trade_counts;
  j.stats = stats;
  j.dumps = dumps;
  j.dump_cap = dump_cap;
  pthread_mutex_init(&j.mu, NULL);
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  pthread_t th[256];
  int32_t started = 0;
  for (int32_t t = 1; t < n_threads; ++t)
    if (pthread_create(&th[started], NULL, worker, &j) == 0) started++;
  worker(&j);
  for (int32_t t = 0; t < started; ++t) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&j.mu);
  return j.failed ? -1 : 0;
}
