// lob_api.cpp -- the C ABI of liblob (declared in include/lob.h): argument checks,
// device memory of a context, choice of kernel form and launch geometry.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lob.h"
#include "lob_internal.h"

#include "lob_ctx.h"

namespace {

thread_local std::string g_create_error;

// Scratch of lob_exec_step_noalloc: agent-order staging [LOB_NOALLOC_MAX_BOOKS][4][8]
// int32, then step bookkeeping [LOB_NOALLOC_MAX_BOOKS][2] int64 -- 2.25 MiB in the
// library's device image, one copy per GPU, held until the process ends.  Host code
// uses it only through the address hipGetSymbolAddress gives for each device.
constexpr size_t kScratchActsBytes = sizeof(int32_t) * 4 * lob::kMsgFields * LOB_NOALLOC_MAX_BOOKS;
constexpr size_t kScratchBytes = kScratchActsBytes + sizeof(int64_t) * 2 * LOB_NOALLOC_MAX_BOOKS;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// The device address of `scratch` on the current device (once per device), or
// nullptr with the error in *err.
void *scratch_on_current_device(std::string *err) {
  static std::mutex mu;
  static std::vector<void *> addr;
  static std::vector<int> state;  // 0 not looked up, 1 found, -1 failed
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
    *err = "no current device";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(mu);
  if ((size_t)dev >= addr.size()) {
    addr.resize(dev + 1, nullptr);
    state.resize(dev + 1, 0);
  }
  if (state[dev] == 0) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    state[dev] = (e == hipSuccess && p) ? 1 : -1;
    addr[dev] = state[dev] == 1 ? p : nullptr;
    if (state[dev] < 0) (void)hipGetLastError();
  }
  if (state[dev] < 0) *err = "the address of the static scratch array could not be found on this device";
  return addr[dev];
}

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

lob_status fail(lob_ctx *c, lob_status st, const std::string &msg) {
  if (c) c->err = msg;
  return st;
}

lob_status hip_fail(lob_ctx *c, hipError_t e, const char *what) {
  return fail(c, LOB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int round_up(int v, int m) { return (v + m - 1) / m * m; }

void free_ctx(lob_ctx *c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(c->d_hdr);
  (void)hipFree(c->d_books);
  (void)hipFree(c->d_log);
  (void)hipFree(c->d_stage);
  (void)hipFree(c->d_exec_acts);
  (void)hipFree(c->d_exec_aux);
  if (c->h_stage) (void)hipHostFree(c->h_stage);
  if (c->ev_staged) (void)hipEventDestroy(c->ev_staged);
  if (c->ev_ragged_done) (void)hipEventDestroy(c->ev_ragged_done);
  if (c->side_stream) (void)hipStreamDestroy(c->side_stream);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  delete c;
}

lob_status check_list(lob_ctx *c, int32_t n) {
  if (!c) return LOB_EINVAL;
  if (n < 0 || n > c->n_books) return fail(c, LOB_EINVAL, "n_books out of range");
  return LOB_OK;
}

// LDS words (int2) one wave of the LDS kernel needs for a window of W slots per
// side: 3 pair arrays per side.
int lds_int2_per_wave(int W) { return 6 * W; }

struct Geometry {
  int W;
  bool spill;
  int bpb;
  int per_wave;
};

// Window and books-per-block for one launch over books of capacity <= cap_limit.
lob_status geometry(lob_ctx *c, int window, int cap_limit, int bpb_want, Geometry *g) {
  int W = std::min(window, cap_limit);
  if (W < 1) W = 1;
  int bpb = std::max(1, std::min(16, bpb_want));
  int per_wave = lds_int2_per_wave(W);
  while (bpb > 1 && (size_t)bpb * per_wave * sizeof(int2) > c->max_lds) --bpb;
  if ((size_t)per_wave * sizeof(int2) > c->max_lds) return fail(c, LOB_ECAP, "LDS window does not fit");
  g->W = W;
  g->spill = cap_limit > W;
  g->bpb = bpb;
  g->per_wave = per_wave;
  return LOB_OK;
}

// One matching launch over books of capacity <= cap_limit: the register kernel when
// the plan allows it and every such book fits in registers, else the LDS kernel.
lob_status launch(lob_ctx *c, lob::ProcArgs a, int window, int cap_limit, int bpb, hipStream_t s) {
  if (a.n == 0) return LOB_OK;
  // waves sharing SIMDs: the register kernel rotates their issue priorities.  Measured
  // on uniform books: a gain at 2 to 4 waves per SIMD, and for steps (short fixed
  // windows) at 8; a loss for long streams at 8 or more waves per SIMD.  One wave per
  // SIMD has nothing to share.
  {
    const int64_t simds = 4 * (int64_t)c->num_cus, n = a.n;
    const bool step = a.msgs && !a.offs && !a.ranges;  // fixed windows of w1 messages
    a.rotate = (a.prio_len == 0 && n > simds && (n <= 4 * simds || step)) ? 1 : 0;
  }
  a.tail_shallow = c->plan.tail_shallow;
  if (c->plan.layout == 1) {  // the paper's unsorted arrays, whole book in LDS
    const int per_wave = (lob::unsorted_lds_ints(cap_limit) + 1) / 2;
    int b = std::max(1, std::min(16, bpb));
    while (b > 1 && (size_t)b * per_wave * sizeof(int2) > c->max_lds) --b;
    if ((size_t)per_wave * sizeof(int2) > c->max_lds) return fail(c, LOB_ECAP, "book does not fit in LDS");
    a.bpb = b;
    a.lds_int2_per_wave = per_wave;
    hipError_t e = lob::launch_process_unsorted(a, s);
    return e == hipSuccess ? LOB_OK : hip_fail(c, e, "process launch");
  }
  // the register kernel's forms with a tail or per-message L2 (but the execution
  // step's level-1 rows) leave a book whose times go backwards to the LDS engine,
  // launched right after them
  auto deferred = [&](lob::ProcArgs b) -> lob_status {
    hipError_t e = lob::launch_process_deferred(b, std::min(cap_limit, 64), s);
    return e == hipSuccess ? LOB_OK : hip_fail(c, e, "deferred launch");
  };
  if (c->plan.registers) {
    if (cap_limit <= lob::small_book_slots()) {  // whole books in registers
      a.bpb = std::max(1, std::min(16, bpb));
      hipError_t e = lob::launch_process_small(a, false, s);
      if (e != hipSuccess) return hip_fail(c, e, "process launch");
      return lob::small_defers(a, false) ? deferred(a) : LOB_OK;
    }
    // the first 128 orders per side in registers, the rest in an LDS tail of
    // 16-byte entries (P, Q, OID, handle), tw per side
    const int tw = (cap_limit - lob::small_book_slots() + 1) & ~1;
    const int per_wave = 4 * tw;
    if ((size_t)per_wave * sizeof(int2) <= c->max_lds) {
      int b = std::max(1, std::min(16, bpb));
      while (b > 1 && (size_t)b * per_wave * sizeof(int2) > c->max_lds) --b;
      a.W = tw;
      a.bpb = b;
      a.lds_int2_per_wave = per_wave;
      hipError_t e = lob::launch_process_small(a, true, s);
      if (e != hipSuccess) return hip_fail(c, e, "process launch");
      return deferred(a);
    }
  }
  Geometry g;
  lob_status st = geometry(c, window, cap_limit, bpb, &g);
  if (st != LOB_OK) return st;
  a.W = g.W;
  a.bpb = g.bpb;
  a.lds_int2_per_wave = g.per_wave;
  hipError_t e = lob::launch_process(a, g.spill, s);
  return e == hipSuccess ? LOB_OK : hip_fail(c, e, "process launch");
}

// The capacity bound of a lob_process_messages / lob_step / lob_exec_step launch:
// the plan's, else the context's largest.
int plan_cap_limit(const lob_ctx *c) {
  return c->plan.max_capacity > 0 ? std::min(c->plan.max_capacity, c->max_cap) : c->max_cap;
}

lob_status run_process(lob_ctx *c, const lob::ProcArgs &a, hipStream_t s) {
  return launch(c, a, c->plan.lds_slots, plan_cap_limit(c), c->plan.books_per_block, s);
}


// One execution step (lob_exec_step) with its agent-order staging acts [n][4][8] and
// step bookkeeping aux [n][2] at the given device addresses.
lob_status exec_step_with(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, const int32_t *window, int32_t W,
                          const int32_t *action_qty, const lob_exec_params *params, lob_exec_state *state,
                          int32_t *obs, double *reward, int32_t *agent_fills, int32_t F, int32_t *agent_fill_counts,
                          int32_t *acts, int64_t *aux, void *stream) {
  if (W < 1 || W > 256) return fail(ctx, LOB_EINVAL, "W out of 1..256");
  if (F < 1) return fail(ctx, LOB_EINVAL, "F < 1");
  if (!params) return fail(ctx, LOB_EINVAL, "params is NULL");
  if (n_books == 0) return LOB_OK;
  if (!window || !aligned16(window)) return fail(ctx, LOB_EINVAL, "window NULL or not 16-byte aligned");
  if (!action_qty || !state || !obs || !reward || !agent_fills || !agent_fill_counts)
    return fail(ctx, LOB_EINVAL, "a buffer is NULL");
  if ((reinterpret_cast<uintptr_t>(obs) & 3) || (reinterpret_cast<uintptr_t>(reward) & 7) ||
      (reinterpret_cast<uintptr_t>(state) & 7))
    return fail(ctx, LOB_EINVAL, "obs / reward / state misaligned");
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = lob::launch_exec_prepare(ctx->d_hdr, ctx->d_books, book_ids, n_books, ctx->n_books, window, W,
                                          action_qty, *params, state, acts, aux, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "exec prepare");
  // the matcher: data then agent orders; level-1 row of every data message into the
  // first 4W ints of the book's observation row; trades logged for the reward
  lob::ProcArgs a = lob::base_args(ctx, book_ids, n_books);
  a.msgs = window;
  a.w1 = W;
  a.msgs2 = acts;
  a.w2 = 4;
  a.l2_mode = LOB_L2_PER_MESSAGE;
  a.levels = 1;
  a.l2_out = obs;
  a.l2_stride = 6 * (int64_t)W + 8;
  a.fills = agent_fills;
  a.fill_cap = F;
  a.fill_counts = agent_fill_counts;
  a.agent_tid = params->agent_tid;
  lob_status st = run_process(ctx, a, s);
  if (st != LOB_OK) return st;
  e = lob::launch_exec_finish(ctx->d_hdr, book_ids, n_books, ctx->n_books, ctx->d_log, window, W, *params, state, obs,
                              reward, agent_fills, F, agent_fill_counts, aux, s);
  return e == hipSuccess ? LOB_OK : hip_fail(ctx, e, "exec finish");
}

}  // namespace

namespace lob {
ProcArgs base_args(lob_ctx *c, const int32_t *ids, int32_t n) {
  ProcArgs a;
  std::memset(&a, 0, sizeof(a));
  a.hdr = c->d_hdr;
  a.books = c->d_books;
  a.books_half = c->books_half;
  a.log = c->d_log;
  a.book_ids = ids;
  a.n = n;
  a.n_total = c->n_books;
  a.levels = c->L;
  return a;
}
lob_status launch_with_plan(lob_ctx *c, const ProcArgs &a, hipStream_t s) { return run_process(c, a, s); }
lob_status launch_with_cap(lob_ctx *c, const ProcArgs &a, int cap_limit, hipStream_t s) {
  return launch(c, a, c->plan.lds_slots, std::max(1, std::min(cap_limit, c->max_cap)), c->plan.books_per_block, s);
}
lob_status set_error(lob_ctx *c, lob_status st, const std::string &msg) { return fail(c, st, msg); }
}  // namespace lob

extern "C" {

lob_status lob_create(const lob_config *cfg, lob_ctx **out) {
  if (!out) return LOB_EINVAL;
  *out = nullptr;
  g_create_error.clear();
  auto bad = [](const char *m) {
    g_create_error = m;
    return LOB_EINVAL;
  };
  if (!cfg) return bad("cfg is NULL");
  if (cfg->n_books < 1) return bad("n_books < 1");
  if (!cfg->capacity_host) return bad("capacity_host is NULL");
  if (cfg->l2_levels < 1 || cfg->l2_levels > LOB_MAX_LEVELS) return bad("l2_levels out of range");
  if (!cfg->trade_log_records_host && cfg->trade_log_default < 0) return bad("trade_log_default < 0");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev)
    return bad("no such HIP device");
  lob_ctx *c = new lob_ctx();
  c->device = cfg->device;
  c->n_books = cfg->n_books;
  c->L = cfg->l2_levels;
  c->caps.assign(cfg->capacity_host, cfg->capacity_host + cfg->n_books);
  std::vector<lob::BookHdr> hdr(cfg->n_books);
  int64_t book_int2 = 0, log_rec = 0;
  for (int i = 0; i < cfg->n_books; ++i) {
    const int cap = c->caps[i];
    if (cap < 1 || cap > LOB_MAX_CAPACITY) {
      delete c;
      return bad("capacity out of range");
    }
    const int64_t lc = cfg->trade_log_records_host ? cfg->trade_log_records_host[i] : cfg->trade_log_default;
    if (lc < 0) {
      delete c;
      return bad("negative trade log size");
    }
    c->max_cap = std::max(c->max_cap, cap);
    lob::BookHdr &h = hdr[i];
    std::memset(&h, 0, sizeof(h));
    h.cap = cap;
    h.book_off = book_int2;
    h.log_off = log_rec;
    h.log_cap = lc;
    book_int2 += 6LL * cap;
    log_rec += lc;
  }
  DeviceGuard g(c->device);
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, c->device);
  if (e != hipSuccess || !g.ok) {
    g_create_error = "hipGetDeviceProperties failed";
    delete c;
    return LOB_EDEVICE;
  }
  c->num_cus = prop.multiProcessorCount;
  c->max_lds = prop.sharedMemPerBlock;
  if (prop.maxSharedMemoryPerMultiProcessor > 0)
    c->max_lds = std::min<size_t>(c->max_lds, prop.maxSharedMemoryPerMultiProcessor);
  if (c->max_lds == 0) c->max_lds = 65536;
  auto alloc = [&](void **p, size_t bytes) {
    return hipMalloc(p, std::max<size_t>(bytes, 256)) == hipSuccess;
  };
  c->stage_bytes = sizeof(int32_t) * 2 * (size_t)c->n_books + sizeof(int64_t) * 2 * (size_t)c->n_books + 256;
  c->books_half = book_int2;
  bool ok = alloc((void **)&c->d_hdr, sizeof(lob::BookHdr) * hdr.size()) &&
            alloc((void **)&c->d_books, sizeof(int2) * 2 * (size_t)book_int2) &&
            alloc((void **)&c->d_log, sizeof(int32_t) * lob::kTradeFields * (size_t)log_rec) &&
            alloc((void **)&c->d_stage, c->stage_bytes) &&
            alloc((void **)&c->d_exec_acts, sizeof(int32_t) * 4 * 8 * (size_t)c->n_books) &&
            alloc((void **)&c->d_exec_aux, sizeof(int64_t) * 2 * (size_t)c->n_books) &&
            hipHostMalloc((void **)&c->h_stage, c->stage_bytes, hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    g_create_error = "device allocation failed";
    free_ctx(c);
    return LOB_ENOMEM;
  }
  e = hipMemcpy(c->d_hdr, hdr.data(), sizeof(lob::BookHdr) * hdr.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_staged, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_ragged_done, hipEventDisableTiming);
  if (e == hipSuccess) c->scratch = scratch_on_current_device(&c->scratch_err);
  if (e == hipSuccess) {  // advisory on this platform
    (void)lob::set_process_lds_limit(c->max_lds);
    (void)lob::set_process_unsorted_lds_limit(c->max_lds);
    (void)lob::set_process_small_lds_limit(c->max_lds);
    (void)hipGetLastError();  // an attribute the platform refuses must not linger as the last error
  }
  if (e != hipSuccess) {
    g_create_error = std::string("context setup: ") + hipGetErrorString(e);
    free_ctx(c);
    return LOB_EDEVICE;
  }
  // default plan: books of capacity <= 128 wholly in registers; larger books in LDS
  // when they fit comfortably, otherwise a 256-slot window with the rest in HBM;
  // four books per workgroup; ragged calls in one launch, longest stream first
  c->plan.lds_slots = c->max_cap <= 1024 ? c->max_cap : 256;
  c->plan.books_per_block = 4;
  c->plan.ragged_split = 0;
  c->plan.lds_slots_big = c->plan.lds_slots;  // (a valid plan: lob_set_plan accepts it back)
  c->plan.ragged_order = 1;
  c->plan.books_per_block_big = 1;
  c->plan.registers = 1;
  *out = c;
  return LOB_OK;
}

void lob_destroy(lob_ctx *ctx) { free_ctx(ctx); }

const char *lob_last_error(const lob_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

lob_status lob_info(const lob_ctx *ctx, int32_t *n_books, int32_t *max_capacity, int32_t *l2_levels) {
  if (!ctx) return LOB_EINVAL;
  if (n_books) *n_books = ctx->n_books;
  if (max_capacity) *max_capacity = ctx->max_cap;
  if (l2_levels) *l2_levels = ctx->L;
  return LOB_OK;
}

lob_status lob_set_plan(lob_ctx *ctx, const lob_plan *plan) {
  if (!ctx || !plan) return LOB_EINVAL;
  if (plan->lds_slots < 1 || plan->lds_slots > LOB_MAX_CAPACITY) return fail(ctx, LOB_EINVAL, "lds_slots");
  if (plan->books_per_block < 1 || plan->books_per_block > 16) return fail(ctx, LOB_EINVAL, "books_per_block");
  if (plan->ragged_split < 0 || plan->ragged_split > LOB_MAX_CAPACITY) return fail(ctx, LOB_EINVAL, "ragged_split");
  if (plan->lds_slots_big < 1 || plan->lds_slots_big > LOB_MAX_CAPACITY)
    return fail(ctx, LOB_EINVAL, "lds_slots_big");
  if (plan->ragged_order != 0 && plan->ragged_order != 1) return fail(ctx, LOB_EINVAL, "ragged_order");
  if (plan->books_per_block_big < 1 || plan->books_per_block_big > 16)
    return fail(ctx, LOB_EINVAL, "books_per_block_big");
  if (plan->registers != 0 && plan->registers != 1) return fail(ctx, LOB_EINVAL, "registers");
  if (plan->layout != 0 && plan->layout != 1) return fail(ctx, LOB_EINVAL, "layout");
  if (plan->max_capacity < 0 || plan->max_capacity > LOB_MAX_CAPACITY) return fail(ctx, LOB_EINVAL, "max_capacity");
  if (plan->tail_shallow != 0 && plan->tail_shallow != 1) return fail(ctx, LOB_EINVAL, "tail_shallow");
  if (plan->layout == 1 && (size_t)lob::unsorted_lds_ints(ctx->max_cap) * sizeof(int32_t) > ctx->max_lds)
    return fail(ctx, LOB_ECAP, "layout 1: the largest book does not fit in LDS");
  for (int w : {plan->lds_slots, plan->lds_slots_big, plan->ragged_split > 0 ? plan->ragged_split : 1})
    if ((size_t)lds_int2_per_wave(std::min(w, ctx->max_cap)) * sizeof(int2) >
        ctx->max_lds)
      return fail(ctx, LOB_ECAP, "LDS window does not fit in LDS");
  ctx->plan = *plan;
  return LOB_OK;
}

lob_status lob_get_plan(const lob_ctx *ctx, lob_plan *plan) {
  if (!ctx || !plan) return LOB_EINVAL;
  *plan = ctx->plan;
  return LOB_OK;
}

lob_status lob_process_messages(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, const int32_t *msgs,
                                const int64_t *msg_offsets, int32_t l2_mode, int32_t *l2_out, void *stream) {
  lob_status st = check_list(ctx, n_books);
  if (st != LOB_OK) return st;
  if (n_books == 0) return LOB_OK;
  if (!msgs || !msg_offsets) return fail(ctx, LOB_EINVAL, "msgs / msg_offsets is NULL");
  if (!aligned16(msgs)) return fail(ctx, LOB_EINVAL, "msgs must be 16-byte aligned");
  if (l2_mode < LOB_L2_NONE || l2_mode > LOB_L2_FINAL) return fail(ctx, LOB_EINVAL, "l2_mode");
  if (l2_mode != LOB_L2_NONE && !l2_out) return fail(ctx, LOB_EINVAL, "l2_out is NULL");
  DeviceGuard g(ctx->device);
  lob::ProcArgs a = lob::base_args(ctx, book_ids, n_books);
  a.msgs = msgs;
  a.offs = msg_offsets;
  a.l2_mode = l2_mode;
  a.l2_out = l2_out;
  return run_process(ctx, a, (hipStream_t)stream);
}

// The pinned staging buffer is rewritten only after the copy of the previous
// schedule out of it has completed.
static lob_status stage_wait(lob_ctx *ctx) {
  if (!ctx->staged_pending) return LOB_OK;
  hipError_t e = hipEventSynchronize(ctx->ev_staged);
  if (e != hipSuccess) return hip_fail(ctx, e, "staging wait");
  ctx->staged_pending = false;
  return LOB_OK;
}

// Copy the first `bytes` of the staging buffer to the device schedule.  The device
// copy is reused: the copy waits for the kernels of the previous ragged call,
// whichever stream it was issued on.
static lob_status stage_copy(lob_ctx *ctx, size_t bytes, hipStream_t s) {
  hipError_t e;
  if (ctx->ragged_pending && (e = hipStreamWaitEvent(s, ctx->ev_ragged_done, 0)) != hipSuccess)
    return hip_fail(ctx, e, "ragged order");
  if ((e = hipMemcpyAsync(ctx->d_stage, ctx->h_stage, bytes, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_fail(ctx, e, "staging copy");
  if ((e = hipEventRecord(ctx->ev_staged, s)) != hipSuccess) return hip_fail(ctx, e, "staging event");
  ctx->staged_pending = true;
  return LOB_OK;
}

// v (list positions in increasing order) sorted by decreasing stream length, equal
// lengths in increasing position: a stable least-significant-digit radix sort of
// (longest - length), 11 bits per pass (two passes for streams below 4M messages).
// The host does this before every ragged launch while the GPU waits, so it is kept
// linear: a comparison sort of 10,000 books took about 0.5 ms.
static void sort_longest_first(std::vector<int32_t> &v, const int64_t *offs) {
  const size_t n = v.size();
  if (n < 2) return;
  int64_t longest = 0;
  for (int32_t i : v) longest = std::max<int64_t>(longest, offs[i + 1] - offs[i]);
  std::vector<uint64_t> key(n), key2(n);
  std::vector<int32_t> v2(n);
  for (size_t k = 0; k < n; ++k) key[k] = (uint64_t)(longest - (offs[v[k] + 1] - offs[v[k]]));
  constexpr int kBits = 11;
  constexpr uint64_t kMask = (1u << kBits) - 1;
  std::vector<uint32_t> count((size_t)1 << kBits);
  for (int shift = 0; shift < 64 && ((uint64_t)longest >> shift) != 0; shift += kBits) {
    std::fill(count.begin(), count.end(), 0u);
    for (size_t k = 0; k < n; ++k) ++count[(key[k] >> shift) & kMask];
    uint32_t sum = 0;
    for (uint32_t &c : count) {
      const uint32_t t = c;
      c = sum;
      sum += t;
    }
    for (size_t k = 0; k < n; ++k) {
      const uint32_t at = count[(key[k] >> shift) & kMask]++;
      key2[at] = key[k];
      v2[at] = v[k];
    }
    key.swap(key2);
    v.swap(v2);
  }
}

lob_status lob_process_ragged(lob_ctx *ctx, const int32_t *book_ids_host, int32_t n_books, const int32_t *msgs,
                              const int64_t *msg_offsets_host, int32_t l2_mode, int32_t *l2_out, void *stream) {
  lob_status st = check_list(ctx, n_books);
  if (st != LOB_OK) return st;
  if (n_books == 0) return LOB_OK;
  if (!msgs || !msg_offsets_host) return fail(ctx, LOB_EINVAL, "msgs / msg_offsets_host is NULL");
  if (!aligned16(msgs)) return fail(ctx, LOB_EINVAL, "msgs must be 16-byte aligned");
  if (l2_mode < LOB_L2_NONE || l2_mode > LOB_L2_FINAL) return fail(ctx, LOB_EINVAL, "l2_mode");
  if (l2_mode != LOB_L2_NONE && !l2_out) return fail(ctx, LOB_EINVAL, "l2_out is NULL");
  const lob_plan &p = ctx->plan;
  // host-side schedule: validate ids, split into capacity buckets, order each bucket
  std::vector<char> seen(ctx->n_books, 0);
  std::vector<int32_t> small, big;
  small.reserve(n_books);
  for (int32_t i = 0; i < n_books; ++i) {
    const int32_t b = book_ids_host ? book_ids_host[i] : i;
    if (b < 0 || b >= ctx->n_books) return fail(ctx, LOB_EINVAL, "book id out of range");
    if (seen[b]) return fail(ctx, LOB_EINVAL, "book id listed twice");
    seen[b] = 1;
    if (msg_offsets_host[i + 1] < msg_offsets_host[i]) return fail(ctx, LOB_EINVAL, "offsets decrease");
    if (p.ragged_split > 0 && ctx->caps[b] > p.ragged_split)
      big.push_back(i);
    else
      small.push_back(i);
  }
  auto len = [&](int32_t i) { return msg_offsets_host[i + 1] - msg_offsets_host[i]; };
  if (p.ragged_order) {
    sort_longest_first(small, msg_offsets_host);
    sort_longest_first(big, msg_offsets_host);
  }
  // stage [ids | rows | ranges] in pinned memory, one copy to the device
  DeviceGuard g(ctx->device);
  hipError_t e;
  if ((st = stage_wait(ctx)) != LOB_OK) return st;
  int32_t *h_ids = ctx->h_stage;
  int32_t *h_rows = h_ids + n_books;
  int64_t *h_ranges = reinterpret_cast<int64_t *>(ctx->h_stage + 2 * (size_t)n_books);  // 8n bytes: aligned
  int32_t k = 0;
  for (const std::vector<int32_t> *v : {&small, &big})
    for (int32_t i : *v) {
      h_ids[k] = book_ids_host ? book_ids_host[i] : i;
      h_rows[k] = i;
      h_ranges[2 * k] = msg_offsets_host[i];
      h_ranges[2 * k + 1] = msg_offsets_host[i + 1];
      ++k;
    }
  const size_t bytes = reinterpret_cast<char *>(h_ranges + 2 * (size_t)n_books) - reinterpret_cast<char *>(h_ids);
  hipStream_t s = (hipStream_t)stream;
  if ((st = stage_copy(ctx, bytes, s)) != LOB_OK) return st;
  const int32_t *d_ids = ctx->d_stage;
  const int32_t *d_rows = d_ids + n_books;
  const int64_t *d_ranges =
      reinterpret_cast<const int64_t *>(ctx->d_stage + 2 * (size_t)n_books);
  lob::ProcArgs a = lob::base_args(ctx, d_ids, (int32_t)small.size());
  a.msgs = msgs;
  a.ranges = d_ranges;
  {
    int64_t longest = 0;
    for (int32_t i = 0; i < n_books; ++i) longest = std::max<int64_t>(longest, len(i));
    a.prio_len = std::max<int64_t>(1, longest / 2);
  }
  a.out_rows = d_rows;
  a.l2_mode = l2_mode;
  a.l2_out = l2_out;
  auto done = [&](lob_status r) -> lob_status {
    if (r != LOB_OK) return r;
    hipError_t ee = hipEventRecord(ctx->ev_ragged_done, s);
    if (ee != hipSuccess) return hip_fail(ctx, ee, "ragged done event");
    ctx->ragged_pending = true;
    return LOB_OK;
  };
  // each launch is sized for the largest capacity among the books it holds
  auto max_cap_of = [&](const std::vector<int32_t> &v) {
    int m = 1;
    for (int32_t i : v) m = std::max(m, (int)ctx->caps[book_ids_host ? book_ids_host[i] : i]);
    return m;
  };
  const int cap_small = max_cap_of(small);
  if (big.empty())
    return done(launch(ctx, a, p.ragged_split > 0 ? p.ragged_split : p.lds_slots, cap_small, p.books_per_block, s));
  // two buckets: the large-capacity launch on the side stream, forked from and
  // joined back into the caller's stream
  lob::ProcArgs b = a;
  b.book_ids = d_ids + small.size();
  b.out_rows = d_rows + small.size();
  b.ranges = d_ranges + 2 * small.size();
  b.n = (int32_t)big.size();
  if ((e = hipEventRecord(ctx->ev_fork, s)) != hipSuccess) return hip_fail(ctx, e, "fork");
  if ((e = hipStreamWaitEvent(ctx->side_stream, ctx->ev_fork, 0)) != hipSuccess) return hip_fail(ctx, e, "fork");
  if ((st = launch(ctx, b, p.lds_slots_big, max_cap_of(big), p.books_per_block_big, ctx->side_stream)) != LOB_OK)
    return st;
  if ((st = launch(ctx, a, p.ragged_split, cap_small, p.books_per_block, s)) != LOB_OK) return st;
  if ((e = hipEventRecord(ctx->ev_join, ctx->side_stream)) != hipSuccess) return hip_fail(ctx, e, "join");
  if ((e = hipStreamWaitEvent(s, ctx->ev_join, 0)) != hipSuccess) return hip_fail(ctx, e, "join");
  return done(LOB_OK);
}

lob_status lob_autotune_ragged(lob_ctx *ctx, const int32_t *book_ids_host, int32_t n_books, const int32_t *msgs,
                               const int64_t *msg_offsets_host, int32_t max_trials, lob_plan *best,
                               float *best_ms, void *stream) {
  lob_status st = check_list(ctx, n_books);
  if (st != LOB_OK) return st;
  if (!best || max_trials < 1 || n_books < 1) return fail(ctx, LOB_EINVAL, "best / max_trials / n_books");
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard g(ctx->device);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(ctx, LOB_EDEVICE, "autotune events");
  const lob_plan base = ctx->plan;
  // the listed books are the first n ints of the device schedule after a ragged
  // call (in launch order), which is what the resets below use
  auto reset_listed = [&]() -> lob_status {
    hipError_t e = lob::launch_reset(ctx->d_hdr, ctx->d_stage, n_books, ctx->n_books, s);
    return e == hipSuccess ? LOB_OK : hip_fail(ctx, e, "autotune reset");
  };
  int trials = 0;
  float best_t = 1e30f;
  lob_plan best_p = base;
  // a candidate's time: the slowest of three runs after an untimed one.  Some plans
  // are bimodal from run to run (the two bucket launches race for the GPU's wave
  // slots, and the longest book can start late); ranking by the worst run favours
  // plans that are fast every time.
  auto trial = [&](lob_plan p) -> lob_status {
    if (trials >= max_trials) return LOB_OK;
    if (lob_set_plan(ctx, &p) != LOB_OK) return LOB_OK;  // candidate does not fit: skip it
    ++trials;
    if (hipEventRecord(e0, s) != hipSuccess) return fail(ctx, LOB_EDEVICE, "autotune event");
    lob_status r = lob_process_ragged(ctx, book_ids_host, n_books, msgs, msg_offsets_host, LOB_L2_NONE, nullptr,
                                      stream);  // stages the schedule; warms caches
    if (r != LOB_OK) return r;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      return fail(ctx, LOB_EDEVICE, "autotune sync");
    {
      // a candidate whose untimed run already took twice the best time is not run again
      float ms0 = 0.f;
      (void)hipEventElapsedTime(&ms0, e0, e1);
      if (ms0 > 2.f * best_t) return reset_listed();
    }
    float t[3];
    for (float &ms : t) {
      if ((r = reset_listed()) != LOB_OK) return r;
      if (hipEventRecord(e0, s) != hipSuccess) return fail(ctx, LOB_EDEVICE, "autotune event");
      r = lob_process_ragged(ctx, book_ids_host, n_books, msgs, msg_offsets_host, LOB_L2_NONE, nullptr, stream);
      if (r != LOB_OK) return r;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return fail(ctx, LOB_EDEVICE, "autotune sync");
      ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
    }
    if ((r = reset_listed()) != LOB_OK) return r;
    const float ms = std::max(t[0], std::max(t[1], t[2]));
    if (ms < best_t) {
      best_t = ms;
      best_p = p;
    }
    return LOB_OK;
  };
  // distinct capacities among the listed books (candidate bucket boundaries)
  std::vector<int32_t> caps;
  for (int32_t i = 0; i < n_books; ++i) {
    const int32_t b = book_ids_host ? book_ids_host[i] : i;
    if (b < 0 || b >= ctx->n_books) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return fail(ctx, LOB_EINVAL, "book id out of range");
    }
    caps.push_back(ctx->caps[b]);
  }
  std::sort(caps.begin(), caps.end());
  caps.erase(std::unique(caps.begin(), caps.end()), caps.end());
  const int maxc = caps.back();
  // the untimed first run of the first candidate starts from empty books too: stage
  // the listed ids where reset_listed reads them and reset the books
  lob_status r = stage_wait(ctx);
  if (r == LOB_OK) {
    for (int32_t i = 0; i < n_books; ++i) ctx->h_stage[i] = book_ids_host ? book_ids_host[i] : i;
    r = stage_copy(ctx, sizeof(int32_t) * (size_t)n_books, s);
  }
  if (r == LOB_OK) r = reset_listed();
  if (r != LOB_OK) goto out;
  // stage 1: structure -- one launch with whole books in LDS or a small window,
  // or two buckets split at each listed capacity below the largest
  {
    lob_plan p = base;
    p.ragged_order = 1;
    p.ragged_split = 0;
    p.books_per_block = 4;
    p.books_per_block_big = 1;
    for (int w : {maxc, 128}) {
      p.lds_slots = std::min(w, maxc);
      if ((r = trial(p)) != LOB_OK) goto out;
    }
    for (size_t k = 0; k + 1 < caps.size(); ++k) {
      p.lds_slots = std::min(128, maxc);
      p.ragged_split = caps[k];
      for (int wb : {maxc, 256}) {
        p.lds_slots_big = std::min(wb, maxc);
        if ((r = trial(p)) != LOB_OK) goto out;
      }
    }
    // the other residencies in one launch: the LDS engine alone, and the paper's
    // unsorted arrays (skipped when the largest book does not fit in LDS)
    lob_plan q = base;
    q.ragged_order = 1;
    q.ragged_split = 0;
    q.books_per_block = 4;
    q.lds_slots = std::min(128, maxc);
    q.registers = 0;
    if ((r = trial(q)) != LOB_OK) goto out;
    q.registers = base.registers;
    q.layout = 1;
    if ((r = trial(q)) != LOB_OK) goto out;
  }
  // stage 1b: the TAIL form's code for drained books, when the batch has books above
  // 128 orders per side
  if (maxc > lob::small_book_slots()) {
    lob_plan p = best_p;
    p.tail_shallow = 1 - p.tail_shallow;
    if ((r = trial(p)) != LOB_OK) goto out;
  }
  // stage 2: books per workgroup of each launch
  {
    const lob_plan s1 = best_p;
    for (int bpb : {1, 2, 8}) {
      lob_plan p = s1;
      p.books_per_block = bpb;
      if ((r = trial(p)) != LOB_OK) goto out;
    }
    if (s1.ragged_split > 0)
      for (int bb : {2, 4}) {
        lob_plan p = best_p;
        p.books_per_block_big = bb;
        if ((r = trial(p)) != LOB_OK) goto out;
      }
  }
  // stage 3: LDS window of the launch that can spill
  {
    const lob_plan s2 = best_p;
    for (int w : {64, 256, 512}) {
      lob_plan p = s2;
      if (p.ragged_split > 0)
        p.lds_slots_big = std::min(w, maxc);
      else
        p.lds_slots = std::min(w, maxc);
      if ((r = trial(p)) != LOB_OK) goto out;
    }
  }

out:
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (r != LOB_OK) {
    ctx->plan = base;
    return r;
  }
  ctx->plan = best_p;
  *best = best_p;
  if (best_ms) *best_ms = best_t;
  return LOB_OK;
}

lob_status lob_step(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, const int32_t *window, int32_t W,
                    const int32_t *actions, int32_t A, int32_t agent_tid, int32_t *l2_out, int32_t *agent_fills,
                    int32_t F, int32_t *agent_fill_counts, void *stream) {
  lob_status st = check_list(ctx, n_books);
  if (st != LOB_OK) return st;
  if (W < 0 || A < 0 || F < 0) return fail(ctx, LOB_EINVAL, "negative W / A / F");
  if (n_books == 0) return LOB_OK;
  if (W > 0 && (!window || !aligned16(window))) return fail(ctx, LOB_EINVAL, "window NULL or not 16-byte aligned");
  if (A > 0 && (!actions || !aligned16(actions))) return fail(ctx, LOB_EINVAL, "actions NULL or not aligned");
  if (!l2_out) return fail(ctx, LOB_EINVAL, "l2_out is NULL");
  if (F > 0 && (!agent_fills || !agent_fill_counts)) return fail(ctx, LOB_EINVAL, "agent_fills is NULL");
  DeviceGuard g(ctx->device);
  lob::ProcArgs a = lob::base_args(ctx, book_ids, n_books);
  a.log = nullptr;
  a.msgs = W > 0 ? window : nullptr;
  a.w1 = W;
  a.msgs2 = A > 0 ? actions : nullptr;
  a.w2 = A;
  a.l2_mode = LOB_L2_FINAL;
  a.l2_out = l2_out;
  a.fills = F > 0 ? agent_fills : nullptr;
  a.fill_cap = F;
  a.fill_counts = F > 0 ? agent_fill_counts : nullptr;
  a.agent_tid = agent_tid;
  return run_process(ctx, a, (hipStream_t)stream);
}

lob_status lob_exec_step(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, const int32_t *window,
                         int32_t W, const int32_t *action_qty, const lob_exec_params *params,
                         lob_exec_state *state, int32_t *obs, double *reward, int32_t *agent_fills, int32_t F,
                         int32_t *agent_fill_counts, void *stream) {
  lob_status st = check_list(ctx, n_books);
  if (st != LOB_OK) return st;
  return exec_step_with(ctx, book_ids, n_books, window, W, action_qty, params, state, obs, reward, agent_fills, F,
                        agent_fill_counts, ctx->d_exec_acts, ctx->d_exec_aux, stream);
}

lob_status lob_exec_step_noalloc(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, const int32_t *window,
                                 int32_t W, const int32_t *action_qty, const lob_exec_params *params,
                                 lob_exec_state *state, int32_t *obs, double *reward, int32_t *agent_fills, int32_t F,
                                 int32_t *agent_fill_counts, void *stream) {
  lob_status st = check_list(ctx, n_books);
  if (st != LOB_OK) return st;
  if (n_books > LOB_NOALLOC_MAX_BOOKS)
    return fail(ctx, LOB_ECAP, "lob_exec_step_noalloc: more than LOB_NOALLOC_MAX_BOOKS (16384) books in one call");
  if (!ctx->scratch) return fail(ctx, LOB_EDEVICE, "lob_exec_step_noalloc: " + ctx->scratch_err);
  int32_t *acts = reinterpret_cast<int32_t *>(ctx->scratch);
  int64_t *aux = reinterpret_cast<int64_t *>(static_cast<unsigned char *>(ctx->scratch) + kScratchActsBytes);
  return exec_step_with(ctx, book_ids, n_books, window, W, action_qty, params, state, obs, reward, agent_fills, F,
                        agent_fill_counts, acts, aux, stream);
}

lob_status lob_read_l2(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, int32_t *l2_out, void *stream) {
  lob_status st = check_list(ctx, n_books);
  if (st != LOB_OK) return st;
  if (n_books == 0) return LOB_OK;
  if (!l2_out) return fail(ctx, LOB_EINVAL, "l2_out is NULL");
  DeviceGuard g(ctx->device);
  hipError_t e = lob::launch_read_l2(ctx->d_hdr, ctx->d_books, book_ids, n_books, ctx->n_books, ctx->L, l2_out,
                                     (hipStream_t)stream);
  return e == hipSuccess ? LOB_OK : hip_fail(ctx, e, "read_l2");
}

lob_status lob_read_trades(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, int32_t *out,
                           int64_t max_records, int64_t *counts, int64_t *offsets, void *stream) {
  lob_status st = check_list(ctx, n_books);
  if (st != LOB_OK) return st;
  if (max_records < 0) return fail(ctx, LOB_EINVAL, "max_records < 0");
  if (!offsets || (n_books > 0 && !counts)) return fail(ctx, LOB_EINVAL, "counts / offsets is NULL");
  if (max_records > 0 && !out) return fail(ctx, LOB_EINVAL, "out is NULL");
  DeviceGuard g(ctx->device);
  hipError_t e = lob::launch_read_trades(ctx->d_hdr, ctx->d_log, book_ids, n_books, ctx->n_books, out, max_records, counts,
                                         offsets, (hipStream_t)stream);
  return e == hipSuccess ? LOB_OK : hip_fail(ctx, e, "read_trades");
}

lob_status lob_read_status(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, lob_book_status *out,
                           void *stream) {
  lob_status st = check_list(ctx, n_books);
  if (st != LOB_OK) return st;
  if (n_books == 0) return LOB_OK;
  if (!out) return fail(ctx, LOB_EINVAL, "out is NULL");
  DeviceGuard g(ctx->device);
  hipError_t e = lob::launch_status(ctx->d_hdr, book_ids, n_books, ctx->n_books, out, (hipStream_t)stream);
  return e == hipSuccess ? LOB_OK : hip_fail(ctx, e, "read_status");
}

lob_status lob_read_book(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, int32_t *out, int32_t dump_cap,
                         void *stream) {
  lob_status st = check_list(ctx, n_books);
  if (st != LOB_OK) return st;
  if (dump_cap < 1) return fail(ctx, LOB_EINVAL, "dump_cap < 1");
  if (n_books == 0) return LOB_OK;
  if (!out) return fail(ctx, LOB_EINVAL, "out is NULL");
  DeviceGuard g(ctx->device);
  hipError_t e = lob::launch_read_book(ctx->d_hdr, ctx->d_books, book_ids, n_books, ctx->n_books, dump_cap, out,
                                       (hipStream_t)stream);
  return e == hipSuccess ? LOB_OK : hip_fail(ctx, e, "read_book");
}

lob_status lob_write_book(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, const int32_t *in,
                          int32_t dump_cap, void *stream) {
  lob_status st = check_list(ctx, n_books);
  if (st != LOB_OK) return st;
  if (dump_cap < 1) return fail(ctx, LOB_EINVAL, "dump_cap < 1");
  if (n_books == 0) return LOB_OK;
  if (!in) return fail(ctx, LOB_EINVAL, "in is NULL");
  DeviceGuard g(ctx->device);
  hipError_t e = lob::launch_write_book(ctx->d_hdr, ctx->d_books, book_ids, n_books, ctx->n_books, dump_cap, in,
                                        (hipStream_t)stream);
  return e == hipSuccess ? LOB_OK : hip_fail(ctx, e, "write_book");
}

lob_status lob_reset(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, void *stream) {
  lob_status st = check_list(ctx, n_books);
  if (st != LOB_OK) return st;
  if (n_books == 0) return LOB_OK;
  DeviceGuard g(ctx->device);
  hipError_t e = lob::launch_reset(ctx->d_hdr, book_ids, n_books, ctx->n_books, (hipStream_t)stream);
  return e == hipSuccess ? LOB_OK : hip_fail(ctx, e, "reset");
}

lob_status lob_seed_l2(lob_ctx *ctx, const int32_t *book_ids, int32_t n_books, const int32_t *l2, int32_t levels,
                       const int32_t *times, int32_t init_tid, void *stream) {
  lob_status st = check_list(ctx, n_books);
  if (st != LOB_OK) return st;
  if (levels < 1 || levels > LOB_MAX_LEVELS) return fail(ctx, LOB_EINVAL, "levels out of range");
  if (n_books == 0) return LOB_OK;
  if (!l2) return fail(ctx, LOB_EINVAL, "l2 is null");
  DeviceGuard g(ctx->device);
  hipError_t e = lob::launch_seed_l2(ctx->d_hdr, ctx->d_books, book_ids, n_books, ctx->n_books, levels, l2, times,
                                     init_tid, (hipStream_t)stream);
  return e == hipSuccess ? LOB_OK : hip_fail(ctx, e, "seed_l2");
}

lob_status lob_selftest(int32_t device, int32_t *out, void *stream) {
  if (!out) return LOB_EINVAL;
  DeviceGuard g(device);
  if (!g.ok) return LOB_EDEVICE;
  if (lob::launch_selftest(out, (hipStream_t)stream) != hipSuccess) return LOB_EDEVICE;
  return lob::launch_selftest_shift(out + 192, (hipStream_t)stream) == hipSuccess ? LOB_OK : LOB_EDEVICE;
}

}  // extern "C"
