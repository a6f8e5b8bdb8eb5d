/*
 * flowgen.h -- seeded synthetic order flow for the batched limit-order-book matcher.
 *
 * Produces message streams shaped like the paper's replay workloads (JAX-LOB,
 * Section 5.1: LOBSTER-style message data, one book per stream): initial resting
 * orders carrying the negative ids of Section 5.1.1, then a mix of limit, cancel,
 * delete and market messages with strictly increasing times.  The inputs are pure
 * bytes; the matcher under test and its oracle both read the same bytes.
 *
 * Randomness: one SplitMix64 stream (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) per (seed, workload tag, book,
 * purpose); normals by Box-Muller; geometric and exponential by inversion.
 *
 * Cancels and deletes must name an order that is still resting, so the generator
 * keeps a small ledger of live orders and updates it for every message it emits
 * (including the fills a crossing order causes).  The ledger only decides which
 * bytes are emitted; no expected value is ever taken from it.
 *
 * Message layout (int32 x 8): {type, side, price, qty, order_id, trader_id,
 * time_s, time_ns}; type 1 limit, 2 cancel, 3 delete, 4 market; side +1 bid,
 * -1 ask.
 */
#ifndef LOB_FLOWGEN_H
#define LOB_FLOWGEN_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Book streams.  Book i (keyed by key_ids[i], or by i when key_ids is NULL) gets
 * 2*seeds_per_side[i] seed limit orders, then n_flow[i] flow messages, written to
 * out + offs[i]*8; offs[i+1]-offs[i] must equal 2*seeds_per_side[i]+n_flow[i].
 * caps[i] is the book's capacity per side (the ledger rejects like the book does).
 * Returns 0, or -1 on bad arguments. */
int32_t fg_generate(uint64_t seed, uint32_t tag, int32_t n_books, const int32_t *key_ids,
                    const int32_t *mids, int32_t tick, const int32_t *caps,
                    const int32_t *seeds_per_side, const int64_t *n_flow, int32_t *out,
                    const int64_t *offs, int32_t n_threads);

/* Agent actions for the environment-step workload: per book and step up to 4
 * orders (type 0 = none), trader id -1, ids from 1e9 upwards per book, limit price
 * mid +/- tick*U{0..5} or market, qty U[1,500], time = times[i][step] (the
 * time of the step's last data message).  out is [n][steps][4][8]. */
int32_t fg_agent(uint64_t seed, uint32_t tag, int32_t n_books, const int32_t *key_ids,
                 const int32_t *mids, int32_t tick, int32_t n_steps, const int32_t *times,
                 int32_t *out, int32_t n_threads);

/* Per-book parameters of the ragged workload: capacity in {50,100,500,1000}
 * (p = .3/.4/.2/.1), flow length floor(exp(U[ln 100, ln 1e5])), mid price
 * U[1e6, 5e7] rounded to a multiple of 100. */
void fg_ragged_params(uint64_t seed, uint32_t tag, int32_t n_books, int32_t *caps,
                      int64_t *n_flow, int32_t *mids);

/* Serving requests: n_req requests with Poisson arrival times (rate lambda per
 * second, in ns from 0), book uniform in [0, n_books), kind 0 replay / 1 step with
 * probability 1/2, size floor(exp(U[0, ln 1000])) messages. */
void fg_requests(uint64_t seed, uint32_t tag, int64_t n_req, double lambda, int32_t n_books,
                 int64_t *arrival_ns, int32_t *book, int32_t *kind, int32_t *size);

#ifdef __cplusplus
}
#endif
#endif
