// lob_ctx.h -- the context object behind the C ABI, shared by the host-side
// sources of liblob (lob_api.cpp, lob_serve.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "lob.h"
#include "lob_internal.h"

namespace lob {
hipError_t launch_process(const ProcArgs &a, bool spill, hipStream_t s);
hipError_t launch_process_deferred(const ProcArgs &a, int W, hipStream_t s);
hipError_t set_process_lds_limit(size_t bytes);
hipError_t launch_reset(BookHdr *hdr, const int32_t *ids, int n, int n_total, hipStream_t s);
hipError_t launch_status(const BookHdr *hdr, const int32_t *ids, int n, int n_total, void *out, hipStream_t s);
hipError_t launch_read_l2(const BookHdr *hdr, int2 *books, const int32_t *ids, int n, int n_total, int L,
                          int32_t *out, hipStream_t s);
hipError_t launch_read_book(const BookHdr *hdr, const int2 *books, const int32_t *ids, int n, int n_total,
                            int dump_cap, int32_t *out, hipStream_t s);
hipError_t launch_write_book(BookHdr *hdr, int2 *books, const int32_t *ids, int n, int n_total, int dump_cap,
                             const int32_t *in, hipStream_t s);
hipError_t launch_read_trades(BookHdr *hdr, const int32_t *log, const int32_t *ids, int n, int n_total,
                              int32_t *out, int64_t max_records, int64_t *counts, int64_t *offsets,
                              hipStream_t s);
hipError_t launch_selftest(int32_t *out, hipStream_t s);
hipError_t launch_exec_prepare(const BookHdr *hdr, const int2 *books, const int32_t *ids, int n, int n_total,
                               const int32_t *window, int W, const int32_t *action_qty, const lob_exec_params &p,
                               lob_exec_state *state, int32_t *acts, int64_t *aux, hipStream_t s);
hipError_t launch_exec_finish(BookHdr *hdr, const int32_t *ids, int n, int n_total, const int32_t *log,
                              const int32_t *window, int W, const lob_exec_params &p, lob_exec_state *state,
                              int32_t *obs, double *reward, const int32_t *fills, int F, const int32_t *fill_counts,
                              const int64_t *aux, hipStream_t s);
hipError_t launch_seed_l2(BookHdr *hdr, int2 *books, const int32_t *ids, int n, int n_total, int L,
                          const int32_t *l2, const int32_t *times, int tid, hipStream_t s);
hipError_t launch_process_small(const ProcArgs &a, bool tail, hipStream_t s);
// Whether that launch leaves books whose times go backwards to k_process_deferred.
bool small_defers(const ProcArgs &a, bool tail);
hipError_t set_process_small_lds_limit(size_t bytes);
hipError_t launch_process_unsorted(const ProcArgs &a, hipStream_t s);
hipError_t set_process_unsorted_lds_limit(size_t bytes);
int unsorted_lds_ints(int cap);
hipError_t launch_selftest_shift(int32_t *out, hipStream_t s);
int small_book_slots();
}  // namespace lob

static_assert(sizeof(lob_book_status) == 96, "lob_book_status layout");

struct lob_ctx {
  int device = 0;
  int n_books = 0, L = 10, max_cap = 0;
  std::vector<int32_t> caps;
  lob::BookHdr *d_hdr = nullptr;
  int2 *d_books = nullptr;  // two buffers per book, books_half int2 apart
  int64_t books_half = 0;
  int32_t *d_log = nullptr;
  lob_plan plan{};
  std::string err;
  int num_cus = 0;
  size_t max_lds = 0;
  // ragged schedule: listed ids, message ranges and output rows of one call, staged
  // in pinned host memory and copied to the device in one transfer
  int32_t *h_stage = nullptr, *d_stage = nullptr;
  size_t stage_bytes = 0;
  hipEvent_t ev_staged = nullptr;  // the last staging copy has completed
  bool staged_pending = false;
  hipEvent_t ev_ragged_done = nullptr;  // all work of the last ragged call
  bool ragged_pending = false;
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // execution steps: the agent orders of each listed book [n_books][4][8] and where
  // its trades of the step start in its log, with its trade count [n_books][2]
  int32_t *d_exec_acts = nullptr;
  int64_t *d_exec_aux = nullptr;
  // device address of the library's static scratch on this context's device
  // (lob_exec_step_noalloc), or nullptr with the reason
  void *scratch = nullptr;
  std::string scratch_err;
};


namespace lob {
// Launch the matching kernel over a.n listed books with the context's plan (or the
// given window / books per workgroup); defined in lob_api.cpp.
lob_status launch_with_plan(lob_ctx *c, const ProcArgs &a, hipStream_t s);
// The same over books whose capacities are at most cap_limit (known on the host).
lob_status launch_with_cap(lob_ctx *c, const ProcArgs &a, int cap_limit, hipStream_t s);
lob_status set_error(lob_ctx *c, lob_status st, const std::string &msg);
ProcArgs base_args(lob_ctx *c, const int32_t *ids, int32_t n);
}  // namespace lob
