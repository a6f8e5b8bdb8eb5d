"""Python binding of liblob (include/lob.h).

Argument marshalling only: every step of the matching path runs in the HIP
kernels of liblob.so.  torch provides device memory (tensors) and streams.
The library must be built (paper_2308_13289_amd.build); without it every call
raises LobError -- there is no fallback.
"""
import ctypes
import os

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblob.so")

OK, EINVAL, ENOMEM, EDEVICE, ECAP = 0, -1, -2, -3, -6
L2_NONE, L2_PER_MESSAGE, L2_FINAL = 0, 1, 2
MAX_CAPACITY, MAX_LEVELS = 4096, 64  # orders per side per book, L2 depth
NOALLOC_MAX_BOOKS = 16384  # books per lob_exec_step_noalloc call
BOOK_SIDE_FULL, BOOK_TIME_ORDER, BOOK_TRADE_FULL, BOOK_FILLS_FULL, BOOK_BAD_LOAD = 1, 2, 4, 8, 16

STATUS_DTYPE = np.dtype([(n, np.int64) for n in (
    "n_msgs", "n_trades", "limit_qty", "market_qty", "traded_qty", "cancelled_qty",
    "market_discarded", "rejected_qty", "cancel_miss")] + [
    ("flags", np.int32), ("n_ask", np.int32), ("n_bid", np.int32), ("pad", np.int32),
    ("log_records", np.int64)])
assert STATUS_DTYPE.itemsize == 96


# execution environment (lob_exec_state / lob_exec_params in lob.h)
EXEC_STATE_DTYPE = np.dtype([("task_side", np.int32), ("task_qty", np.int32), ("exec_qty", np.int32),
                             ("done", np.int32), ("revenue", np.int64), ("p_init", np.int32),
                             ("start_s", np.int32), ("start_ns", np.int32), ("end_s", np.int32),
                             ("next_oid", np.int32), ("flags", np.int32)])
assert EXEC_STATE_DTYPE.itemsize == 48
EXEC_TRADES_MISSING = 1
EXEC_FILLS_MISSING = 2


class ExecParams(ctypes.Structure):
    _fields_ = [("tick", ctypes.c_int32), ("passive_ticks", ctypes.c_int32), ("agent_tid", ctypes.c_int32),
                ("keep_trades", ctypes.c_int32), ("lam", ctypes.c_double)]


class LobError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"liblob status {status}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("n_books", ctypes.c_int32), ("capacity_host", ctypes.POINTER(ctypes.c_int32)),
                ("l2_levels", ctypes.c_int32), ("device", ctypes.c_int32),
                ("trade_log_records_host", ctypes.POINTER(ctypes.c_int64)),
                ("trade_log_default", ctypes.c_int64), ("flags", ctypes.c_uint32)]


class Plan(ctypes.Structure):
    _fields_ = [("lds_slots", ctypes.c_int32), ("books_per_block", ctypes.c_int32),
                ("ragged_split", ctypes.c_int32), ("lds_slots_big", ctypes.c_int32),
                ("ragged_order", ctypes.c_int32), ("books_per_block_big", ctypes.c_int32),
                ("registers", ctypes.c_int32), ("layout", ctypes.c_int32), ("max_capacity", ctypes.c_int32),
                ("tail_shallow", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


_lib = None
EXPORTS = ["lob_create", "lob_destroy", "lob_last_error", "lob_info", "lob_set_plan", "lob_get_plan",
           "lob_process_messages", "lob_process_ragged", "lob_autotune_ragged", "lob_step", "lob_read_l2", "lob_read_trades", "lob_read_status",
           "lob_read_book", "lob_write_book", "lob_reset", "lob_seed_l2", "lob_selftest", "lob_windows",
           "lob_exec_step", "lob_exec_step_noalloc"]


def load(path=None):
    """Load liblob.so and declare its signatures (no GPU is touched)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise LobError(EINVAL, f"{p} is not built (python -m paper_2308_13289_amd.build)")
    L = ctypes.CDLL(p)
    vp, i32, i64, P32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)
    L.lob_create.restype = i32
    L.lob_create.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(vp)]
    L.lob_destroy.restype = None
    L.lob_destroy.argtypes = [vp]
    L.lob_last_error.restype = ctypes.c_char_p
    L.lob_last_error.argtypes = [vp]
    L.lob_info.restype = i32
    L.lob_info.argtypes = [vp, P32, P32, P32]
    L.lob_set_plan.restype = i32
    L.lob_set_plan.argtypes = [vp, ctypes.POINTER(Plan)]
    L.lob_get_plan.restype = i32
    L.lob_get_plan.argtypes = [vp, ctypes.POINTER(Plan)]
    L.lob_process_messages.restype = i32
    L.lob_process_messages.argtypes = [vp, vp, i32, vp, vp, i32, vp, vp]
    L.lob_process_ragged.restype = i32
    L.lob_process_ragged.argtypes = [vp, vp, i32, vp, vp, i32, vp, vp]
    L.lob_autotune_ragged.restype = i32
    L.lob_autotune_ragged.argtypes = [vp, vp, i32, vp, vp, i32, ctypes.POINTER(Plan),
                                      ctypes.POINTER(ctypes.c_float), vp]
    L.lob_step.restype = i32
    L.lob_step.argtypes = [vp, vp, i32, vp, i32, vp, i32, i32, vp, vp, i32, vp, vp]
    L.lob_read_l2.restype = i32
    L.lob_read_l2.argtypes = [vp, vp, i32, vp, vp]
    L.lob_read_trades.restype = i32
    L.lob_read_trades.argtypes = [vp, vp, i32, vp, i64, vp, vp, vp]
    L.lob_read_status.restype = i32
    L.lob_read_status.argtypes = [vp, vp, i32, vp, vp]
    L.lob_read_book.restype = i32
    L.lob_read_book.argtypes = [vp, vp, i32, vp, i32, vp]
    L.lob_write_book.restype = i32
    L.lob_write_book.argtypes = [vp, vp, i32, vp, i32, vp]
    L.lob_reset.restype = i32
    L.lob_reset.argtypes = [vp, vp, i32, vp]
    L.lob_exec_step.restype = i32
    L.lob_exec_step.argtypes = [vp, vp, i32, vp, i32, vp, ctypes.POINTER(ExecParams), vp, vp, vp, vp, i32, vp, vp]
    L.lob_exec_step_noalloc.restype = i32
    L.lob_exec_step_noalloc.argtypes = L.lob_exec_step.argtypes
    L.lob_windows.restype = i32
    L.lob_windows.argtypes = [vp, i64, i32, i32, i32, i32, i32, vp, vp, vp]
    L.lob_seed_l2.restype = i32
    L.lob_seed_l2.argtypes = [vp, vp, i32, vp, i32, vp, i32, vp]
    L.lob_selftest.restype = i32
    L.lob_selftest.argtypes = [i32, vp, vp]
    if path is None:
        _lib = L
    return L


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream, device):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def windows(msgs, start_s, window_s, msgs_per_step, max_steps, n_windows):
    """Windowed replay data of one book's stream (host numpy [n][8] int32): returns
    (windows [n_windows][max_steps][msgs_per_step][8], steps [n_windows],
    first [n_windows + 1]).  Raises LobError if a window needs more steps."""
    m = np.ascontiguousarray(msgs, dtype=np.int32).reshape(-1, 8)
    out = np.zeros((n_windows, max_steps, msgs_per_step, 8), np.int32)
    steps = np.zeros(n_windows, np.int32)
    first = np.zeros(n_windows + 1, np.int64)
    st = load().lob_windows(m.ctypes.data if len(m) else None, len(m), int(start_s), int(window_s),
                            int(msgs_per_step), int(max_steps), int(n_windows), out.ctypes.data,
                            steps.ctypes.data, first.ctypes.data)
    if st != OK:
        raise LobError(st, "lob_windows: " + ("a window needs more than max_steps steps" if st == ECAP
                                              else "bad arguments or times out of order"))
    return out, steps, first


def selftest(device=0):
    out = torch.empty(576, dtype=torch.int32, device=f"cuda:{device}")
    st = load().lob_selftest(device, _ptr(out), _stream(None, out.device))
    if st != OK:
        raise LobError(st, "selftest launch failed")
    return out


class Context:
    """A set of books resident on one GPU (lob_create / lob_destroy)."""

    def __init__(self, capacities, l2_levels=10, device=0, trade_log_records=None,
                 trade_log_default=0):
        self._lib = load()
        caps = np.ascontiguousarray(capacities, dtype=np.int32)
        self.capacities = caps
        self.device = torch.device(f"cuda:{device}")
        self.levels = int(l2_levels)
        cfg = Config()
        cfg.n_books = caps.shape[0]
        cfg.capacity_host = caps.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        cfg.l2_levels = self.levels
        cfg.device = device
        self._logs = None
        if trade_log_records is not None:
            logs = np.asarray(trade_log_records, dtype=np.int64)
            if logs.ndim == 0:
                logs = np.full(caps.shape[0], int(logs), np.int64)
            if logs.shape != caps.shape:
                raise ValueError("trade_log_records: one entry per book (or one for all)")
            self._logs = np.ascontiguousarray(logs)
            cfg.trade_log_records_host = self._logs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        cfg.trade_log_default = int(trade_log_default)
        cfg.flags = 0
        h = ctypes.c_void_p()
        st = self._lib.lob_create(ctypes.byref(cfg), ctypes.byref(h))
        if st != OK:
            raise LobError(st, self._lib.lob_last_error(None).decode())
        self._h = h
        self.n_books = int(caps.shape[0])

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lob_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, st):
        if st != OK:
            raise LobError(st, self._lib.lob_last_error(self._h).decode())

    def _ids(self, book_ids, n):
        if book_ids is None:
            return None, (self.n_books if n is None else int(n))
        return _ptr(book_ids, torch.int32, "book_ids"), int(book_ids.numel())

    # -- plan
    def get_plan(self):
        p = Plan()
        self._check(self._lib.lob_get_plan(self._h, ctypes.byref(p)))
        return p

    def set_plan(self, **kw):
        p = self.get_plan()
        names = {f for f, _ in Plan._fields_}
        for k, v in kw.items():
            if k not in names:
                raise KeyError(f"lob_plan has no field {k!r}")
            setattr(p, k, int(v))
        self._check(self._lib.lob_set_plan(self._h, ctypes.byref(p)))
        return p

    # -- matching
    def process(self, msgs, offsets, book_ids=None, l2_mode=L2_NONE, l2_out=None, stream=None):
        ids, n = self._ids(book_ids, offsets.numel() - 1)
        self._check(self._lib.lob_process_messages(
            self._h, ids, n, _ptr(msgs, torch.int32, "msgs"), _ptr(offsets, torch.int64, "offsets"),
            l2_mode, _ptr(l2_out, torch.int32, "l2_out"), _stream(stream, self.device)))

    def process_ragged(self, msgs, offsets_host, book_ids_host=None, l2_mode=L2_NONE, l2_out=None,
                       stream=None):
        """Ragged batch: offsets (and book ids) are host arrays; the library orders and
        buckets the books (see lob_plan)."""
        offs = np.ascontiguousarray(offsets_host, dtype=np.int64)
        n = offs.shape[0] - 1
        ids = None
        if book_ids_host is not None:
            ids = np.ascontiguousarray(book_ids_host, dtype=np.int32)
            if ids.shape[0] != n:
                raise ValueError("book_ids_host and offsets_host disagree")
        self._check(self._lib.lob_process_ragged(
            self._h, None if ids is None else ctypes.c_void_p(ids.ctypes.data), n,
            _ptr(msgs, torch.int32, "msgs"), ctypes.c_void_p(offs.ctypes.data), l2_mode,
            _ptr(l2_out, torch.int32, "l2_out"), _stream(stream, self.device)))

    def autotune_ragged(self, msgs, offsets_host, book_ids_host=None, max_trials=24, stream=None):
        """Pick (and install) the fastest plan for this ragged batch; resets the
        listed books.  Returns (plan dict, best time in ms)."""
        offs = np.ascontiguousarray(offsets_host, dtype=np.int64)
        n = offs.shape[0] - 1
        ids = None if book_ids_host is None else np.ascontiguousarray(book_ids_host, dtype=np.int32)
        best = Plan()
        ms = ctypes.c_float()
        self._check(self._lib.lob_autotune_ragged(
            self._h, None if ids is None else ctypes.c_void_p(ids.ctypes.data), n,
            _ptr(msgs, torch.int32, "msgs"), ctypes.c_void_p(offs.ctypes.data), int(max_trials),
            ctypes.byref(best), ctypes.byref(ms), _stream(stream, self.device)))
        return best.as_dict(), float(ms.value)

    def step(self, window, l2_out, actions=None, book_ids=None, agent_tid=-1, fills=None,
             fill_counts=None, stream=None):
        n = window.shape[0]
        ids, n = self._ids(book_ids, n)
        W = window.shape[1]
        A = 0 if actions is None else actions.shape[1]
        F = 0 if fills is None else fills.shape[1]
        self._check(self._lib.lob_step(
            self._h, ids, n, _ptr(window, torch.int32, "window"), W,
            _ptr(actions, torch.int32, "actions"), A, agent_tid, _ptr(l2_out, torch.int32, "l2_out"),
            _ptr(fills, torch.int32, "fills"), F, _ptr(fill_counts, torch.int32, "fill_counts"),
            _stream(stream, self.device)))

    # -- readouts
    def read_l2(self, book_ids=None, out=None, stream=None):
        ids, n = self._ids(book_ids, None)
        if out is None:
            out = torch.empty((n, 2, self.levels, 2), dtype=torch.int32, device=self.device)
        self._check(self._lib.lob_read_l2(self._h, ids, n, _ptr(out, torch.int32, "out"),
                                          _stream(stream, self.device)))
        return out

    def read_trades(self, max_records, book_ids=None, out=None, stream=None):
        """Returns (records [max_records, 6], counts [n], offsets [n+1]) device tensors."""
        ids, n = self._ids(book_ids, None)
        if out is None:
            out = torch.empty((max(int(max_records), 1), 6), dtype=torch.int32, device=self.device)
        counts = torch.empty(max(n, 1), dtype=torch.int64, device=self.device)
        offsets = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        self._check(self._lib.lob_read_trades(
            self._h, ids, n, _ptr(out, torch.int32, "out"), int(max_records), _ptr(counts), _ptr(offsets),
            _stream(stream, self.device)))
        return out, counts[:n], offsets

    def read_status(self, book_ids=None, stream=None):
        """numpy structured array (STATUS_DTYPE) of per-book counters; synchronizes."""
        ids, n = self._ids(book_ids, None)
        buf = torch.empty(max(n, 1) * STATUS_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        self._check(self._lib.lob_read_status(self._h, ids, n, _ptr(buf), _stream(stream, self.device)))
        return buf.cpu().numpy()[:n * STATUS_DTYPE.itemsize].view(STATUS_DTYPE)

    def read_book(self, dump_cap=None, book_ids=None, out=None, stream=None):
        ids, n = self._ids(book_ids, None)
        dump_cap = int(dump_cap or self.capacities.max())
        if out is None:
            out = torch.empty((n, 2, dump_cap, 6), dtype=torch.int32, device=self.device)
        self._check(self._lib.lob_read_book(self._h, ids, n, _ptr(out, torch.int32, "out"), dump_cap,
                                            _stream(stream, self.device)))
        return out

    def write_book(self, dump, book_ids=None, stream=None):
        ids, n = self._ids(book_ids, dump.shape[0])
        self._check(self._lib.lob_write_book(self._h, ids, n, _ptr(dump, torch.int32, "dump"),
                                             int(dump.shape[2]), _stream(stream, self.device)))

    def reset(self, book_ids=None, stream=None):
        ids, n = self._ids(book_ids, None)
        self._check(self._lib.lob_reset(self._h, ids, n, _stream(stream, self.device)))

    def exec_step(self, window, action_qty, state, obs, reward, fills, fill_counts, tick=100, passive_ticks=1,
                  agent_tid=-1, keep_trades=False, lam=0.0, book_ids=None, stream=None, noalloc=False):
        """Execution-environment step (lob_exec_step, or lob_exec_step_noalloc with
        noalloc=True): window[n][W][8], action_qty[n][4] int32, state = uint8 device
        tensor of n * 48 bytes (EXEC_STATE_DTYPE), obs [n][6W+8] int32, reward [n]
        float64, fills [n][F][6], fill_counts [n]."""
        ids, n = self._ids(book_ids, window.shape[0])
        p = ExecParams(int(tick), int(passive_ticks), int(agent_tid), int(bool(keep_trades)), float(lam))
        fn = self._lib.lob_exec_step_noalloc if noalloc else self._lib.lob_exec_step
        self._check(fn(
            self._h, ids, n, _ptr(window, torch.int32, "window"), int(window.shape[1]),
            _ptr(action_qty, torch.int32, "action_qty"), ctypes.byref(p), _ptr(state, torch.uint8, "state"),
            _ptr(obs, torch.int32, "obs"), _ptr(reward, torch.float64, "reward"), _ptr(fills, torch.int32, "fills"),
            int(fills.shape[1]), _ptr(fill_counts, torch.int32, "fill_counts"), _stream(stream, self.device)))

    def seed_l2(self, l2, times=None, init_tid=0, book_ids=None, stream=None):
        """Start books from L2 snapshots l2[n][2][levels][2] (device int32); times[n][2]
        device int32 or None."""
        ids, n = self._ids(book_ids, l2.shape[0])
        self._check(self._lib.lob_seed_l2(self._h, ids, n, _ptr(l2, torch.int32, "l2"), int(l2.shape[2]),
                                          _ptr(times, torch.int32, "times"), int(init_tid),
                                          _stream(stream, self.device)))
