// lob_serve.cpp -- the request loop of liblob (lob_server_* in include/lob.h).
//
// Continuous batching over the books of one context:
//   queue      requests in arrival order (FIFO)
//   admission  a request joins the batch being formed only if its book has no
//              request on the device and no earlier request still queued (so a
//              book's requests run in arrival order), and if the batch still fits
//              the slot's share of the HBM staging budget
//   slots      n_slots batches in flight, each on its own stream with its own
//              pinned + device staging; a batch = one matching launch (one wave
//              per book: its messages, then its agent orders) over books of one
//              capacity class (<= 128 or larger, so that the launch is sized for
//              its own books), one trade-log drain for its books, one copy of the
//              outputs back to pinned memory
//   retire     when a slot's event has completed, results are copied into the
//              requests' host buffers and their books are free again
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <vector>

#include "lob_ctx.h"

namespace {

constexpr size_t kAlign = 256;
size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int64_t steady_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Byte layout of one batch's staging, identical on host (pinned) and device.
struct Layout {
  // inputs (one host-to-device copy of [0, in_end))
  size_t ranges, ids, actions, msgs, in_end;
  // outputs (one device-to-host copy of [out_begin, out_end))
  size_t l2, fills, fcounts, tcounts, toffs, trades, out_begin, out_end;
};

Layout layout(int32_t n, int64_t n_msgs, int64_t trade_room, int L, int F) {
  Layout y;
  size_t o = 0;
  y.ranges = o;  o = up(o + sizeof(int64_t) * 2 * n);
  y.ids = o;     o = up(o + sizeof(int32_t) * n);
  y.actions = o; o = up(o + sizeof(int32_t) * 4 * 8 * n);
  y.msgs = o;    o = up(o + sizeof(int32_t) * 8 * n_msgs);
  y.in_end = o;
  y.out_begin = o;
  y.l2 = o;      o = up(o + sizeof(int32_t) * 4 * L * n);
  y.fills = o;   o = up(o + sizeof(int32_t) * 6 * (size_t)F * n);
  y.fcounts = o; o = up(o + sizeof(int32_t) * n);
  y.tcounts = o; o = up(o + sizeof(int64_t) * n);
  y.toffs = o;   o = up(o + sizeof(int64_t) * (n + 1));
  y.trades = o;  o = up(o + sizeof(int32_t) * 6 * trade_room);
  y.out_end = o;
  return y;
}

struct Req {
  lob_request r;
  int64_t arrival_ns = 0, launch_ns = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  char *h = nullptr;  // pinned staging
  char *d = nullptr;  // device staging
  size_t bytes = 0;
  bool busy = false;
  std::vector<int64_t> reqs;  // indices into lob_server::table
  Layout y{};
  int64_t trade_room = 0;
};

}  // namespace

struct lob_server {
  lob_ctx *ctx = nullptr;
  lob_server_config cfg{};
  int64_t t0 = 0;
  std::vector<Slot> slots;
  std::vector<Req> table;        // every request ever submitted
  std::deque<int64_t> queue;     // waiting, arrival order
  std::vector<char> on_device;   // per book: a request of it is in flight
  std::vector<int64_t> seen;     // per book: last batch scan that met it
  int64_t scan_id = 0;
  std::deque<lob_completion> ready;
  int64_t max_trade_room = 0;    // per slot
  int64_t max_msgs = 0;          // per slot
};

namespace {

// Worst-case trades of one request: every trade empties a standing order (at most
// the resting orders plus those added by the request) or ends an aggressor.
int64_t trade_bound(const lob_ctx *c, const lob_request &r) {
  return 2LL * c->caps[r.book] + 2LL * (r.n_msgs + r.n_actions);
}

void free_server(lob_server *s) {
  if (!s) return;
  for (Slot &sl : s->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.h) (void)hipHostFree(sl.h);
    if (sl.d) (void)hipFree(sl.d);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  delete s;
}

// Copy a finished batch's results to the requests' buffers.
void retire(lob_server *s, Slot &sl) {
  const lob_ctx *c = s->ctx;
  const Layout &y = sl.y;
  const int L = c->L, F = s->cfg.fill_cap;
  const int64_t now = steady_ns() - s->t0;
  const int32_t *l2 = reinterpret_cast<const int32_t *>(sl.h + y.l2);
  const int32_t *fills = reinterpret_cast<const int32_t *>(sl.h + y.fills);
  const int32_t *fcounts = reinterpret_cast<const int32_t *>(sl.h + y.fcounts);
  const int64_t *tcounts = reinterpret_cast<const int64_t *>(sl.h + y.tcounts);
  const int64_t *toffs = reinterpret_cast<const int64_t *>(sl.h + y.toffs);
  const int32_t *trades = reinterpret_cast<const int32_t *>(sl.h + y.trades);
  for (size_t i = 0; i < sl.reqs.size(); ++i) {
    Req &q = s->table[sl.reqs[i]];
    lob_completion cpl;
    cpl.tag = q.r.tag;
    cpl.status = LOB_OK;
    cpl.arrival_ns = q.arrival_ns;
    cpl.launch_ns = q.launch_ns;
    if (q.r.kind == LOB_REQ_REPLAY) {
      const int64_t n = tcounts[i];
      const int64_t k = std::min<int64_t>(n, q.r.trades_room);
      if (k > 0 && q.r.trades_host) std::memcpy(q.r.trades_host, trades + toffs[i] * 6, sizeof(int32_t) * 6 * k);
      if (k < n) cpl.status = LOB_ECAP;
      cpl.n_out = (int32_t)n;
    } else {
      if (q.r.l2_host) std::memcpy(q.r.l2_host, l2 + (size_t)i * 4 * L, sizeof(int32_t) * 4 * L);
      const int32_t n = fcounts[i];
      const int32_t k = std::min(std::min(n, F), q.r.fills_room);
      if (k > 0 && q.r.fills_host) std::memcpy(q.r.fills_host, fills + (size_t)i * F * 6, sizeof(int32_t) * 6 * k);
      if (k < n) cpl.status = LOB_ECAP;
      cpl.n_out = n;
    }
    cpl.complete_ns = now;
    s->on_device[q.r.book] = 0;
    s->ready.push_back(cpl);
  }
  sl.reqs.clear();
  sl.busy = false;
}

// Form one batch from the queue into a free slot and launch it.
lob_status launch_batch(lob_server *s, Slot &sl) {
  lob_ctx *c = s->ctx;
  // scan a bounded prefix of the queue in arrival order
  const int64_t scan = ++s->scan_id;
  const size_t limit = std::min(s->queue.size(), (size_t)8 * s->cfg.max_batch + 4096);
  std::vector<int64_t> take, keep;
  int64_t msgs = 0, room = 0;
  // one batch holds books of one class -- sides that fit in registers (capacity
  // <= 128) or larger -- so that its single launch takes the form and occupancy of
  // its own books; the class is the first eligible request's
  constexpr int kRegCap = 128;
  int batch_class = -1;
  int cap_bound = 1;
  for (size_t k = 0; k < limit; ++k) {
    const int64_t qi = s->queue.front();
    s->queue.pop_front();
    const lob_request &r = s->table[qi].r;
    const int cls = c->caps[r.book] <= kRegCap ? 0 : 1;
    bool ok = (int32_t)take.size() < s->cfg.max_batch && !s->on_device[r.book] && s->seen[r.book] != scan &&
              (batch_class < 0 || cls == batch_class);
    const int64_t tb = trade_bound(c, r);
    if (ok && (msgs + r.n_msgs > s->max_msgs || room + tb > s->max_trade_room)) ok = false;
    s->seen[r.book] = scan;  // later requests of this book wait for a later batch
    if (ok) {
      take.push_back(qi);
      msgs += r.n_msgs;
      room += tb;
      batch_class = cls;
      cap_bound = std::max(cap_bound, (int)c->caps[r.book]);
    } else {
      keep.push_back(qi);
    }
  }
  // the requests not taken go back to the front, in their order
  for (size_t k = keep.size(); k-- > 0;) s->queue.push_front(keep[k]);
  if (take.empty()) return LOB_OK;
  const int32_t n = (int32_t)take.size();
  sl.y = layout(n, msgs, room, c->L, s->cfg.fill_cap);
  sl.trade_room = room;
  const Layout &y = sl.y;
  int64_t *ranges = reinterpret_cast<int64_t *>(sl.h + y.ranges);
  int32_t *ids = reinterpret_cast<int32_t *>(sl.h + y.ids);
  int32_t *acts = reinterpret_cast<int32_t *>(sl.h + y.actions);
  int32_t *m = reinterpret_cast<int32_t *>(sl.h + y.msgs);
  int64_t pos = 0;
  const int64_t now = steady_ns() - s->t0;
  for (int32_t i = 0; i < n; ++i) {
    Req &q = s->table[take[i]];
    const lob_request &r = q.r;
    ids[i] = r.book;
    ranges[2 * i] = pos;
    ranges[2 * i + 1] = pos + r.n_msgs;
    if (r.n_msgs > 0) std::memcpy(m + pos * 8, r.msgs_host, sizeof(int32_t) * 8 * r.n_msgs);
    pos += r.n_msgs;
    std::memset(acts + (size_t)i * 32, 0, sizeof(int32_t) * 32);
    if (r.kind == LOB_REQ_STEP && r.n_actions > 0)
      std::memcpy(acts + (size_t)i * 32, r.actions_host, sizeof(int32_t) * 8 * r.n_actions);
    q.launch_ns = now;
    s->on_device[r.book] = 1;
  }
  sl.reqs.assign(take.begin(), take.end());
  sl.busy = true;
  hipError_t e = hipMemcpyAsync(sl.d, sl.h, y.in_end, hipMemcpyHostToDevice, sl.stream);
  if (e != hipSuccess) return lob::set_error(c, LOB_EDEVICE, std::string("server upload: ") + hipGetErrorString(e));
  lob::ProcArgs a = lob::base_args(c, reinterpret_cast<const int32_t *>(sl.d + y.ids), n);
  a.msgs = reinterpret_cast<const int32_t *>(sl.d + y.msgs);
  a.ranges = reinterpret_cast<const int64_t *>(sl.d + y.ranges);
  a.msgs2 = reinterpret_cast<const int32_t *>(sl.d + y.actions);
  a.w2 = 4;
  a.l2_mode = LOB_L2_FINAL;
  a.l2_out = reinterpret_cast<int32_t *>(sl.d + y.l2);
  a.fills = reinterpret_cast<int32_t *>(sl.d + y.fills);
  a.fill_cap = s->cfg.fill_cap;
  a.fill_counts = reinterpret_cast<int32_t *>(sl.d + y.fcounts);
  a.agent_tid = s->cfg.agent_tid;
  lob_status st = lob::launch_with_cap(c, a, cap_bound, sl.stream);
  if (st != LOB_OK) return st;
  e = lob::launch_read_trades(c->d_hdr, c->d_log, a.book_ids, n, c->n_books,
                              reinterpret_cast<int32_t *>(sl.d + y.trades), room,
                              reinterpret_cast<int64_t *>(sl.d + y.tcounts),
                              reinterpret_cast<int64_t *>(sl.d + y.toffs), sl.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(sl.h + y.out_begin, sl.d + y.out_begin, y.out_end - y.out_begin, hipMemcpyDeviceToHost,
                       sl.stream);
  if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
  if (e != hipSuccess) return lob::set_error(c, LOB_EDEVICE, std::string("server batch: ") + hipGetErrorString(e));
  return LOB_OK;
}

}  // namespace

extern "C" {

lob_status lob_server_create(lob_ctx *ctx, const lob_server_config *cfg, lob_server **out) {
  if (!ctx || !cfg || !out) return LOB_EINVAL;
  *out = nullptr;
  if (cfg->n_slots < 1 || cfg->n_slots > 16 || cfg->max_batch < 1 || cfg->max_request_msgs < 1 ||
      cfg->fill_cap < 0 || cfg->hbm_budget <= 0)
    return lob::set_error(ctx, LOB_EINVAL, "server config");
  lob_server *s = new lob_server();
  s->ctx = ctx;
  s->cfg = *cfg;
  s->t0 = steady_ns();
  s->on_device.assign(ctx->n_books, 0);
  s->seen.assign(ctx->n_books, -1);
  // per slot: a batch of max_batch requests; messages and trade room sized from the
  // slot's share of the budget
  const size_t share = (size_t)(cfg->hbm_budget / cfg->n_slots);
  const Layout fixed = layout(cfg->max_batch, 0, 0, ctx->L, cfg->fill_cap);
  if (share <= fixed.out_end + 2 * kAlign) {
    delete s;
    return lob::set_error(ctx, LOB_ECAP, "hbm_budget too small for max_batch");
  }
  // bytes per message: 32 in + at most 2 trades * 24 out
  const int64_t per_msg = 32 + 2 * 24;
  s->max_msgs = (int64_t)(share - fixed.out_end - 2 * kAlign) / per_msg;
  s->max_trade_room = 2 * s->max_msgs;
  // every request up to max_request_msgs must fit an empty slot
  const int64_t need_room = 2LL * ctx->max_cap + 2LL * (cfg->max_request_msgs + 4);
  if (s->max_msgs < cfg->max_request_msgs || s->max_trade_room < need_room) {
    delete s;
    return lob::set_error(ctx, LOB_ECAP, "hbm_budget too small for max_request_msgs");
  }
  const size_t bytes = layout(cfg->max_batch, s->max_msgs, s->max_trade_room, ctx->L, cfg->fill_cap).out_end;
  s->slots.resize(cfg->n_slots);
  for (Slot &sl : s->slots) {
    sl.bytes = bytes;
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void **)&sl.h, bytes, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&sl.d, bytes) != hipSuccess) {
      free_server(s);
      return lob::set_error(ctx, LOB_ENOMEM, "server staging allocation");
    }
  }
  *out = s;
  return LOB_OK;
}

void lob_server_destroy(lob_server *srv) { free_server(srv); }

int64_t lob_server_now(const lob_server *srv) { return srv ? steady_ns() - srv->t0 : 0; }

lob_status lob_server_submit(lob_server *srv, const lob_request *req, int64_t arrival_ns) {
  if (!srv || !req) return LOB_EINVAL;
  lob_ctx *c = srv->ctx;
  if (req->book < 0 || req->book >= c->n_books) return lob::set_error(c, LOB_EINVAL, "request book id");
  if (req->kind != LOB_REQ_REPLAY && req->kind != LOB_REQ_STEP) return lob::set_error(c, LOB_EINVAL, "kind");
  if (req->n_msgs < 0 || req->n_msgs > srv->cfg.max_request_msgs || (req->n_msgs > 0 && !req->msgs_host))
    return lob::set_error(c, LOB_EINVAL, "request messages");
  if (req->n_actions < 0 || req->n_actions > 4 || (req->n_actions > 0 && !req->actions_host))
    return lob::set_error(c, LOB_EINVAL, "request actions");
  Req q;
  q.r = *req;
  q.arrival_ns = arrival_ns;
  srv->table.push_back(q);
  srv->queue.push_back((int64_t)srv->table.size() - 1);
  return LOB_OK;
}

lob_status lob_server_poll(lob_server *srv, lob_completion *out, int32_t max_out, int32_t *n_out) {
  if (!srv || (max_out > 0 && !out)) return LOB_EINVAL;
  const int prev_dev = [&] {
    int d = -1;
    (void)hipGetDevice(&d);
    return d;
  }();
  if (prev_dev != srv->ctx->device) (void)hipSetDevice(srv->ctx->device);
  lob_status st = LOB_OK;
  for (Slot &sl : srv->slots) {
    if (!sl.busy) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipSuccess)
      retire(srv, sl);
    else if (q != hipErrorNotReady)
      st = lob::set_error(srv->ctx, LOB_EDEVICE, std::string("server batch failed: ") + hipGetErrorString(q));
  }
  if (st == LOB_OK)
    for (Slot &sl : srv->slots) {
      if (sl.busy || srv->queue.empty()) continue;
      if ((st = launch_batch(srv, sl)) != LOB_OK) break;
    }
  int32_t k = 0;
  while (k < max_out && !srv->ready.empty()) {
    out[k++] = srv->ready.front();
    srv->ready.pop_front();
  }
  if (n_out) *n_out = k;
  if (prev_dev >= 0 && prev_dev != srv->ctx->device) (void)hipSetDevice(prev_dev);
  return st;
}

lob_status lob_server_run(lob_server *srv, const lob_request *reqs, const int64_t *arrival_ns, int64_t n,
                          lob_completion *out) {
  if (!srv || n < 0 || (n > 0 && (!reqs || !arrival_ns || !out))) return LOB_EINVAL;
  const int64_t start = lob_server_now(srv);
  int64_t next = 0, done = 0;
  std::vector<lob_completion> buf(256);
  while (done < n) {
    const int64_t t = lob_server_now(srv) - start;
    while (next < n && arrival_ns[next] <= t) {
      lob_status st = lob_server_submit(srv, &reqs[next], start + arrival_ns[next]);
      if (st != LOB_OK) return st;
      ++next;
    }
    int32_t got = 0;
    lob_status st = lob_server_poll(srv, buf.data(), (int32_t)buf.size(), &got);
    if (st != LOB_OK) return st;
    for (int32_t i = 0; i < got; ++i) out[done++] = buf[i];
  }
  return LOB_OK;
}

}  // extern "C"
