/*
 * flowgen.c -- seeded synthetic order flow (see flowgen.h).
 *
 * Distributions (one stream per book; all draws in the order written below):
 *   seeds     : cap/2 bids at mid - k*tick and cap/2 asks at mid + k*tick with
 *               k = 1 + Geometric(0.3) on {0, 1, ...}; ids -9000, -9001, ...
 *               (the initial-order convention of the paper's Section 5.1.1);
 *               times (34199 s, i ns)
 *   flow      : time starts at (34200 s, 0 ns) and advances by
 *               1 + floor(Exponential(mean 1e6 ns)) per message, carried into
 *               seconds; type by one uniform draw:
 *                 55% limit  side +/-1, price mid + tick*round(N(0, 5^2))
 *                 30% cancel a uniformly chosen live order, qty U[1, resting]
 *                  5% delete a uniformly chosen live order, qty = resting
 *                 10% market side +/-1 (the price field holds an ignored draw)
 *               a cancel or delete with no live order becomes a limit
 *   qty       : 1 + floor(LogNormal(mu 4, sigma 1)), clipped to 10000
 *   ids       : flow orders are numbered 1, 2, ... per book; trader ids U{1..1000}
 */
#include "flowgen.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ SplitMix64 */

typedef struct {
  uint64_t s;
} rng_t;

static uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static uint64_t next64(rng_t *r) {
  r->s += 0x9E3779B97F4A7C15ULL;
  return sm64_mix(r->s);
}

enum { PURPOSE_FLOW = 0x11, PURPOSE_AGENT = 0x22, PURPOSE_PARAMS = 0x33, PURPOSE_REQ = 0x44 };

static rng_t stream_for(uint64_t seed, uint32_t tag, int64_t key, uint32_t purpose) {
  rng_t r;
  uint64_t h = sm64_mix(seed + 0x9E3779B97F4A7C15ULL);
  h = sm64_mix(h ^ ((uint64_t)tag << 32) ^ purpose);
  h = sm64_mix(h ^ (uint64_t)key);
  r.s = h;
  return r;
}

/* uniform in [0, 1) and in (0, 1] with 53 random bits */
static double u01(rng_t *r) { return (double)(next64(r) >> 11) * (1.0 / 9007199254740992.0); }
static double u01c(rng_t *r) { return (double)((next64(r) >> 11) + 1) * (1.0 / 9007199254740992.0); }

/* uniform integer in [0, n), n >= 1, by multiply-shift on 32 random bits */
static int64_t below(rng_t *r, int64_t n) {
  return (int64_t)(((next64(r) >> 32) * (uint64_t)n) >> 32);
}

static double normal01(rng_t *r) { /* Box-Muller, cosine branch */
  double u1 = u01c(r), u2 = u01(r);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

static int32_t geometric(rng_t *r, double p) { /* failures before the first success */
  return (int32_t)floor(log(u01c(r)) / log(1.0 - p));
}

static int32_t draw_qty(rng_t *r) {
  double v = exp(4.0 + normal01(r));
  if (!(v < 9999.0)) return 10000;
  return 1 + (int32_t)floor(v);
}

/* ------------------------------------------------------------- ledger of live orders */

typedef struct {
  int32_t price, qty, oid, tid;
} live_t;

typedef struct {
  live_t *o;
  int32_t n, cap;
} side_t;

typedef struct {
  side_t bid, ask; /* each kept best-first; equal prices in arrival order */
  int32_t cap;
} ledger_t;

static void side_remove(side_t *s, int32_t k) {
  memmove(&s->o[k], &s->o[k + 1], sizeof(live_t) * (size_t)(s->n - k - 1));
  s->n--;
}

static void side_insert(side_t *s, int is_bid, live_t x) {
  int32_t k = 0;
  while (k < s->n && (is_bid ? s->o[k].price >= x.price : s->o[k].price <= x.price)) k++;
  memmove(&s->o[k + 1], &s->o[k], sizeof(live_t) * (size_t)(s->n - k));
  s->o[k] = x;
  s->n++;
}

/* sweep the opposite side; returns the unfilled remainder */
static int32_t sweep(ledger_t *L, int buys, int32_t limit, int32_t q) {
  side_t *opp = buys ? &L->ask : &L->bid;
  while (q > 0 && opp->n > 0) {
    live_t *b = &opp->o[0];
    if (buys ? b->price > limit : b->price < limit) break;
    int32_t f = q < b->qty ? q : b->qty;
    q -= f;
    b->qty -= f;
    if (b->qty == 0) side_remove(opp, 0);
  }
  return q;
}

static void ledger_limit(ledger_t *L, int buys, live_t x) {
  x.qty = sweep(L, buys, x.price, x.qty);
  side_t *own = buys ? &L->bid : &L->ask;
  if (x.qty > 0 && own->n < L->cap) side_insert(own, buys, x);
}

/* ------------------------------------------------------------------ one book */

static void put(int32_t *m, int32_t T, int32_t S, int32_t P, int32_t Q, int32_t oid, int32_t tid,
                int32_t ts, int32_t tns) {
  m[0] = T;
  m[1] = S;
  m[2] = P;
  m[3] = Q;
  m[4] = oid;
  m[5] = tid;
  m[6] = ts;
  m[7] = tns;
}

static int gen_book(uint64_t seed, uint32_t tag, int64_t key, int32_t mid, int32_t tick, int32_t cap,
                    int32_t spb, int64_t n_flow, int32_t *out) {
  ledger_t L;
  L.cap = cap;
  L.bid.n = L.ask.n = 0;
  L.bid.cap = L.ask.cap = cap;
  L.bid.o = (live_t *)malloc(sizeof(live_t) * (size_t)(cap + 1));
  L.ask.o = (live_t *)malloc(sizeof(live_t) * (size_t)(cap + 1));
  if (!L.bid.o || !L.ask.o) {
    free(L.bid.o);
    free(L.ask.o);
    return -1;
  }
  rng_t r = stream_for(seed, tag, key, PURPOSE_FLOW);
  int32_t *m = out;
  for (int32_t i = 0; i < 2 * spb; ++i, m += 8) {
    int buys = i < spb;
    int32_t k = 1 + geometric(&r, 0.3);
    int32_t price = buys ? mid - k * tick : mid + k * tick;
    int32_t q = draw_qty(&r);
    live_t x = {price, q, -9000 - i, 0};
    put(m, 1, buys ? 1 : -1, price, q, x.oid, 0, 34199, i);
    ledger_limit(&L, buys, x);
  }
  int32_t ts = 34200, tns = 0, next_oid = 1;
  for (int64_t j = 0; j < n_flow; ++j, m += 8) {
    if (j > 0) {
      int64_t d = 1 + (int64_t)floor(-1.0e6 * log(u01c(&r)));
      int64_t ns = (int64_t)tns + d;
      ts += (int32_t)(ns / 1000000000LL);
      tns = (int32_t)(ns % 1000000000LL);
    }
    double u = u01(&r);
    int kind = u < 0.55 ? 1 : u < 0.85 ? 2 : u < 0.90 ? 3 : 4;
    int32_t nlive = L.bid.n + L.ask.n;
    if ((kind == 2 || kind == 3) && nlive == 0) kind = 1;
    if (kind == 1 || kind == 4) {
      int buys = u01(&r) < 0.5;
      int32_t price = mid + tick * (int32_t)lround(5.0 * normal01(&r));
      int32_t q = draw_qty(&r);
      int32_t tid = 1 + (int32_t)below(&r, 1000);
      int32_t oid = next_oid++;
      put(m, kind, buys ? 1 : -1, price, q, oid, tid, ts, tns);
      if (kind == 1) {
        live_t x = {price, q, oid, tid};
        ledger_limit(&L, buys, x);
      } else {
        sweep(&L, buys, buys ? INT32_MAX : 0, q);
      }
    } else {
      int32_t k = (int32_t)below(&r, nlive);
      int buys = k < L.bid.n;
      side_t *s = buys ? &L.bid : &L.ask;
      int32_t idx = buys ? k : k - L.bid.n;
      live_t *o = &s->o[idx];
      int32_t q = kind == 3 ? o->qty : 1 + (int32_t)below(&r, o->qty);
      put(m, kind, buys ? 1 : -1, o->price, q, o->oid, o->tid, ts, tns);
      o->qty -= q;
      if (o->qty <= 0) side_remove(s, idx);
    }
  }
  free(L.bid.o);
  free(L.ask.o);
  return 0;
}

/* ------------------------------------------------------------------ threading */

typedef struct {
  int32_t n, next, failed;
  pthread_mutex_t mu;
  void (*fn)(void *ctx, int32_t i, int32_t *failed);
  void *ctx;
} pool_t;

static void *pool_worker(void *arg) {
  pool_t *p = (pool_t *)arg;
  for (;;) {
    pthread_mutex_lock(&p->mu);
    int32_t i = p->next++;
    pthread_mutex_unlock(&p->mu);
    if (i >= p->n) break;
    int32_t f = 0;
    p->fn(p->ctx, i, &f);
    if (f) {
      pthread_mutex_lock(&p->mu);
      p->failed = 1;
      pthread_mutex_unlock(&p->mu);
    }
  }
  return NULL;
}

static int32_t run_pool(int32_t n, int32_t n_threads, void (*fn)(void *, int32_t, int32_t *), void *ctx) {
  pool_t p;
  p.n = n;
  p.next = 0;
  p.failed = 0;
  p.fn = fn;
  p.ctx = ctx;
  pthread_mutex_init(&p.mu, NULL);
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  pthread_t th[256];
  int32_t started = 0;
  for (int32_t t = 1; t < n_threads; ++t)
    if (pthread_create(&th[started], NULL, pool_worker, &p) == 0) started++;
  pool_worker(&p);
  for (int32_t t = 0; t < started; ++t) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&p.mu);
  return p.failed ? -1 : 0;
}

typedef struct {
  uint64_t seed;
  uint32_t tag;
  const int32_t *key_ids, *mids, *caps, *spb;
  int32_t tick;
  const int64_t *n_flow, *offs;
  int32_t *out;
} gen_ctx_t;

static void gen_one(void *vc, int32_t i, int32_t *failed) {
  gen_ctx_t *c = (gen_ctx_t *)vc;
  int64_t key = c->key_ids ? c->key_ids[i] : i;
  if (gen_book(c->seed, c->tag, key, c->mids[i], c->tick, c->caps[i], c->spb[i], c->n_flow[i],
               c->out + (size_t)c->offs[i] * 8) != 0)
    *failed = 1;
}

int32_t fg_generate(uint64_t seed, uint32_t tag, int32_t n_books, const int32_t *key_ids,
                    const int32_t *mids, int32_t tick, const int32_t *caps,
                    const int32_t *seeds_per_side, const int64_t *n_flow, int32_t *out,
                    const int64_t *offs, int32_t n_threads) {
  if (n_books < 0 || !mids || !caps || !seeds_per_side || !n_flow || !offs || (n_books && !out))
    return -1;
  for (int32_t i = 0; i < n_books; ++i) {
    if (caps[i] < 1 || seeds_per_side[i] < 0 || seeds_per_side[i] > caps[i] || n_flow[i] < 0) return -1;
    if (offs[i + 1] - offs[i] != 2 * (int64_t)seeds_per_side[i] + n_flow[i]) return -1;
  }
  gen_ctx_t c = {seed, tag, key_ids, mids, caps, seeds_per_side, tick, n_flow, offs, out};
  return run_pool(n_books, n_threads, gen_one, &c);
}

typedef struct {
  uint64_t seed;
  uint32_t tag;
  const int32_t *key_ids, *mids, *times;
  int32_t tick, n_steps;
  int32_t *out;
} agent_ctx_t;

static void agent_one(void *vc, int32_t i, int32_t *failed) {
  (void)failed;
  agent_ctx_t *c = (agent_ctx_t *)vc;
  int64_t key = c->key_ids ? c->key_ids[i] : i;
  rng_t r = stream_for(c->seed, c->tag, key, PURPOSE_AGENT);
  int32_t next_oid = 1000000000;
  for (int32_t s = 0; s < c->n_steps; ++s) {
    int32_t *m = c->out + ((size_t)i * c->n_steps + s) * 4 * 8;
    const int32_t *t = c->times + ((size_t)i * c->n_steps + s) * 2;
    memset(m, 0, sizeof(int32_t) * 32);
    int32_t n = (int32_t)below(&r, 5);
    for (int32_t k = 0; k < n; ++k) {
      int32_t T = u01(&r) < 0.5 ? 1 : 4;
      int32_t S = u01(&r) < 0.5 ? 1 : -1;
      int32_t sgn = u01(&r) < 0.5 ? 1 : -1;
      int32_t price = c->mids[i] + sgn * c->tick * (int32_t)below(&r, 6);
      int32_t q = 1 + (int32_t)below(&r, 500);
      put(m + 8 * k, T, S, T == 1 ? price : 0, q, next_oid++, -1, t[0], t[1]);
    }
  }
}

int32_t fg_agent(uint64_t seed, uint32_t tag, int32_t n_books, const int32_t *key_ids,
                 const int32_t *mids, int32_t tick, int32_t n_steps, const int32_t *times,
                 int32_t *out, int32_t n_threads) {
  if (n_books < 0 || n_steps < 0 || !mids || !times || !out) return -1;
  agent_ctx_t c = {seed, tag, key_ids, mids, times, tick, n_steps, out};
  return run_pool(n_books, n_threads, agent_one, &c);
}

void fg_ragged_params(uint64_t seed, uint32_t tag, int32_t n_books, int32_t *caps, int64_t *n_flow,
                      int32_t *mids) {
  for (int32_t i = 0; i < n_books; ++i) {
    rng_t r = stream_for(seed, tag, i, PURPOSE_PARAMS);
    double u = u01(&r);
    caps[i] = u < 0.3 ? 50 : u < 0.7 ? 100 : u < 0.9 ? 500 : 1000;
    n_flow[i] = (int64_t)floor(exp(log(100.0) + u01(&r) * (log(1.0e5) - log(100.0))));
    if (n_flow[i] < 100) n_flow[i] = 100;
    if (n_flow[i] > 100000) n_flow[i] = 100000;
    double mid = 1.0e6 + u01(&r) * (5.0e7 - 1.0e6);
    mids[i] = (int32_t)(100 * llround(mid / 100.0));
  }
}

void fg_requests(uint64_t seed, uint32_t tag, int64_t n_req, double lambda, int32_t n_books,
                 int64_t *arrival_ns, int32_t *book, int32_t *kind, int32_t *size) {
  rng_t r = stream_for(seed, tag, 0, PURPOSE_REQ);
  double t = 0.0;
  for (int64_t k = 0; k < n_req; ++k) {
    t += -log(u01c(&r)) / lambda * 1.0e9;
    arrival_ns[k] = (int64_t)t;
    book[k] = (int32_t)below(&r, n_books);
    kind[k] = u01(&r) < 0.5 ? 0 : 1;
    int32_t s = (int32_t)floor(exp(u01(&r) * log(1000.0)));
    size[k] = s < 1 ? 1 : s > 1000 ? 1000 : s;
  }
}
