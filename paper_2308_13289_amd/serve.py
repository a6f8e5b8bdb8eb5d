"""Binding of the liblob request loop (lob_server_* in include/lob.h) and the
serving workload: Poisson arrivals of replay and step requests over books of
mixed capacity, each request carrying the next consecutive slice of its book's
synthetic message stream.

Marshalling only: batching, admission and the matching all run in liblob.
"""
import ctypes

import numpy as np

from . import lob
from . import workload as W

REPLAY, STEP = 0, 1
EXPORTS = ["lob_server_create", "lob_server_destroy", "lob_server_now", "lob_server_submit", "lob_server_poll",
           "lob_server_run"]


class ServerConfig(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int32), ("hbm_budget", ctypes.c_int64), ("max_batch", ctypes.c_int32),
                ("max_request_msgs", ctypes.c_int32), ("fill_cap", ctypes.c_int32),
                ("agent_tid", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int64), ("book", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("msgs_host", ctypes.c_void_p), ("n_msgs", ctypes.c_int32), ("n_actions", ctypes.c_int32),
                ("actions_host", ctypes.c_void_p), ("trades_host", ctypes.c_void_p),
                ("trades_room", ctypes.c_int32), ("l2_host", ctypes.c_void_p), ("fills_host", ctypes.c_void_p),
                ("fills_room", ctypes.c_int32)]


class Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int64), ("status", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("arrival_ns", ctypes.c_int64), ("launch_ns", ctypes.c_int64), ("complete_ns", ctypes.c_int64)]


COMPLETION_DTYPE = np.dtype([("tag", np.int64), ("status", np.int32), ("n_out", np.int32),
                             ("arrival_ns", np.int64), ("launch_ns", np.int64), ("complete_ns", np.int64)])
assert COMPLETION_DTYPE.itemsize == ctypes.sizeof(Completion)

_declared = False


def _lib():
    global _declared
    L = lob.load()
    if not _declared:
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.lob_server_create.restype = i32
        L.lob_server_create.argtypes = [vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
        L.lob_server_destroy.restype = None
        L.lob_server_destroy.argtypes = [vp]
        L.lob_server_now.restype = i64
        L.lob_server_now.argtypes = [vp]
        L.lob_server_submit.restype = i32
        L.lob_server_submit.argtypes = [vp, ctypes.POINTER(Request), i64]
        L.lob_server_poll.restype = i32
        L.lob_server_poll.argtypes = [vp, vp, i32, ctypes.POINTER(i32)]
        L.lob_server_run.restype = i32
        L.lob_server_run.argtypes = [vp, vp, vp, i64, vp]
        _declared = True
    return L


class Server:
    def __init__(self, ctx, n_slots=4, hbm_budget=1 << 30, max_batch=4096, max_request_msgs=1000,
                 fill_cap=64, agent_tid=-1):
        self.ctx = ctx
        self.L = _lib()
        cfg = ServerConfig(n_slots, hbm_budget, max_batch, max_request_msgs, fill_cap, agent_tid)
        h = ctypes.c_void_p()
        st = self.L.lob_server_create(ctx._h, ctypes.byref(cfg), ctypes.byref(h))
        if st != lob.OK:
            raise lob.LobError(st, self.L.lob_last_error(ctx._h).decode())
        self._h = h
        self.cfg = cfg

    def close(self):
        if getattr(self, "_h", None):
            self.L.lob_server_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def run(self, reqs, arrival_ns):
        """Open-loop run of a prepared ServingBatch request array; returns the
        completions (numpy, COMPLETION_DTYPE) in completion order."""
        n = len(reqs)
        arr = np.ascontiguousarray(arrival_ns, dtype=np.int64)
        out = np.zeros(n, COMPLETION_DTYPE)
        st = self.L.lob_server_run(self._h, ctypes.addressof(reqs), arr.ctypes.data, n, out.ctypes.data)
        if st != lob.OK:
            raise lob.LobError(st, self.L.lob_last_error(self.ctx._h).decode())
        return out


class ServingWorkload:
    """Books (capacity mix {50,100,500,1000}, seeded with cap/2 orders per side)
    and a request trace: arrival times, book, kind, the request's message slice
    and, for steps, up to 4 agent orders.  Output buffers for every request."""

    def __init__(self, n_books, lam, duration_s, seed=W.SEED, tag=W.TAGS["c4"], max_msgs=1000, fill_cap=64,
                 levels=10, threads=None):
        n_req_max = int(lam * duration_s * 1.2 + 100)
        arr, book, kind, size = W.requests(n_req_max, lam, n_books, seed=seed, tag=tag)
        keep = arr < int(duration_s * 1e9)
        self.arrival = arr[keep].copy()
        self.book = book[keep].copy()
        self.kind = kind[keep].copy()
        self.size = np.minimum(size[keep], max_msgs).astype(np.int32)
        n = len(self.arrival)
        self.n = n
        caps, _, mids = W.ragged_params(n_books, seed=seed, tag=tag)
        need = np.bincount(self.book, weights=self.size, minlength=n_books).astype(np.int64)
        self.w = W.generate(tag, caps, mids, caps // 2, need, seed=seed, threads=threads, name="serving")
        self.caps, self.levels, self.fill_cap = caps, levels, fill_cap
        # request k of a book takes the next size[k] flow messages of that book
        seeds = 2 * (caps // 2).astype(np.int64)
        cursor = self.w.offs[:-1] + seeds
        self.msg_start = np.zeros(n, np.int64)
        order = np.argsort(self.arrival, kind="stable")
        assert (order == np.arange(n)).all()
        step_idx = np.zeros(n, np.int64)
        n_steps = np.zeros(n_books, np.int64)
        for k in range(n):
            b = self.book[k]
            self.msg_start[k] = cursor[b]
            cursor[b] += self.size[k]
            if self.kind[k] == STEP:
                step_idx[k] = n_steps[b]
                n_steps[b] += 1
        # agent orders of step requests: time = the request's last message time
        max_steps = int(max(1, n_steps.max()))
        times = np.zeros((n_books, max_steps, 2), np.int32)
        st_k = np.nonzero(self.kind == STEP)[0]
        last = self.msg_start[st_k] + self.size[st_k] - 1
        times[self.book[st_k], step_idx[st_k]] = self.w.msgs[last, 6:8]
        acts = W.agent_actions(tag, mids, max_steps, times, seed=seed, threads=threads)
        self.actions = np.zeros((n, 4, 8), np.int32)
        self.actions[st_k] = acts[self.book[st_k], step_idx[st_k]]
        self.n_actions = (self.actions[:, :, 0] != 0).sum(axis=1).astype(np.int32)
        # outputs
        self.trade_room = (2 * caps[self.book] + 2 * (self.size + 4)).astype(np.int64)
        self.trade_offs = np.concatenate([[0], np.cumsum(np.where(self.kind == REPLAY, self.trade_room, 0))])
        self.trades = np.zeros((int(self.trade_offs[-1]) + 1, 6), np.int32)
        self.l2 = np.zeros((n, 2, levels, 2), np.int32)
        self.fills = np.zeros((n, fill_cap, 6), np.int32)
        self._reqs = None

    @property
    def seed_offsets(self):
        return self.w.offs[:-1], self.w.offs[:-1] + 2 * (self.caps // 2)

    def requests(self):
        """ctypes array of lob_request pointing into this object's arrays."""
        n = self.n
        R = (Request * n)()
        mb, ab, tb = self.w.msgs.ctypes.data, self.actions.ctypes.data, self.trades.ctypes.data
        lb, fb = self.l2.ctypes.data, self.fills.ctypes.data
        for k in range(n):
            r = R[k]
            r.tag = k
            r.book = int(self.book[k])
            r.kind = int(self.kind[k])
            r.msgs_host = mb + int(self.msg_start[k]) * 32
            r.n_msgs = int(self.size[k])
            if r.kind == STEP:
                r.n_actions = int(self.n_actions[k])
                r.actions_host = ab + k * 128
                r.l2_host = lb + k * 4 * self.levels * 4
                r.fills_host = fb + k * self.fill_cap * 24
                r.fills_room = self.fill_cap
            else:
                r.trades_host = tb + int(self.trade_offs[k]) * 24
                r.trades_room = int(self.trade_room[k])
        self._reqs = R
        return R

    def oracle_streams(self, books):
        """Each listed book's stream as the server processes it: initial orders, then
        per request (arrival order) its messages and, for a step, its agent orders.
        Returns msgs, offs and per request (index, first, last message index)."""
        parts, offs, spans = [], [0], []
        pos = 0
        by_book = {int(b): [] for b in books}
        for k in range(self.n):
            b = int(self.book[k])
            if b in by_book:
                by_book[b].append(k)
        for b in books:
            b = int(b)
            s0, s1 = self.w.offs[b], self.w.offs[b] + 2 * (self.caps[b] // 2)
            parts.append(self.w.msgs[s0:s1])
            pos += s1 - s0
            for k in by_book[b]:
                m = self.w.msgs[self.msg_start[k]:self.msg_start[k] + self.size[k]]
                a = self.actions[k, :self.n_actions[k]] if self.kind[k] == STEP else np.zeros((0, 8), np.int32)
                first = pos
                parts += [m, a]
                pos += len(m) + len(a)
                spans.append((k, first, pos - 1))
            offs.append(pos)
        return np.concatenate(parts), np.array(offs, np.int64), spans
