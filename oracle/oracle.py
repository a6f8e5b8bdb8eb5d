"""Python view of the reference oracle (lob_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use this module; the product path never imports it.

The oracle is the plain sequential matching engine of JAX-LOB (Frey et al. 2023),
Section 4: unsorted fixed-capacity book sides, a full scan for the best standing
order, and a clean-up pass after every basic operation.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lob_oracle.c")
BUILT = os.path.join(HERE, "liboracle.so")
# tests that plant mistakes in a copy of the oracle point this at the copy
LIB = os.environ.get("LOB_ORACLE_LIB", BUILT)

L2_NONE, L2_PER_MESSAGE, L2_FINAL = 0, 1, 2
FLAG_SIDE_FULL, FLAG_TIME_ORDER, FLAG_TRADE_FULL, FLAG_BAD_LOAD = 1, 2, 4, 16


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "n_msgs", "n_trades", "limit_qty", "market_qty", "traded_qty", "cancelled_qty",
        "market_discarded", "rejected_qty", "cancel_miss")] + [
        ("flags", ctypes.c_int32), ("pad", ctypes.c_int32)]


STATS_DTYPE = np.dtype([(n, np.int64) for n in (
    "n_msgs", "n_trades", "limit_qty", "market_qty", "traded_qty", "cancelled_qty",
    "market_discarded", "rejected_qty", "cancel_miss")] + [("flags", np.int32), ("pad", np.int32)])
assert STATS_DTYPE.itemsize == ctypes.sizeof(Stats)


def build(force=False):
    """Compile liboracle.so with gcc (plain C11, -O3)."""
    if not force and os.path.exists(BUILT) and os.path.getmtime(BUILT) >= max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "lob_oracle.h"))):
        return BUILT
    tmp = BUILT + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                           "-pthread", SRC, "-o", tmp])
    os.replace(tmp, BUILT)
    return BUILT


_lib = None


def lib():
    global _lib
    if _lib is None:
        if LIB == BUILT and not os.path.exists(BUILT):
            build()
        L = ctypes.CDLL(LIB)
        P32, P64, VP = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p
        L.orc_new.restype = VP
        L.orc_new.argtypes = [ctypes.c_int32]
        L.orc_free.argtypes = [VP]
        L.orc_process.restype = ctypes.c_int32
        L.orc_process.argtypes = [VP, P32, P32, ctypes.c_int32]
        L.orc_l2.argtypes = [VP, ctypes.c_int32, P32]
        L.orc_dump.restype = ctypes.c_int32
        L.orc_dump.argtypes = [VP, ctypes.c_int32, P32]
        L.orc_get_stats.argtypes = [VP, ctypes.POINTER(Stats)]
        L.orc_seed_l2.restype = ctypes.c_int32
        L.orc_seed_l2.argtypes = [VP, P32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.orc_run.restype = ctypes.c_int32
        L.orc_run.argtypes = [ctypes.c_int32, P32, P32, P64, ctypes.c_int32, ctypes.c_int32, P32,
                              P32, P64, P64, P64, VP, P32, ctypes.c_int32, ctypes.c_int32]
        _lib = L
    return _lib


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if a is not None else None


def _p64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if a is not None else None


class Book:
    """One book driven message by message (for invariant checks)."""

    def __init__(self, cap):
        self.cap = int(cap)
        self._h = lib().orc_new(self.cap)
        if not self._h:
            raise ValueError("bad capacity")
        self._tr = np.zeros((self.cap, 8), np.int32)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_free(self._h)
            self._h = None

    def process(self, msg):
        m = np.ascontiguousarray(msg, dtype=np.int32)
        n = lib().orc_process(self._h, _p32(m), _p32(self._tr), self.cap)
        return self._tr[:n].copy()

    def seed_l2(self, l2, tid=0, ts=0, tns=0):
        """Empty the book and place one order per present level of an L2 snapshot
        [2][levels][2]; returns the orders placed, or -1 if it is not a book."""
        a = np.ascontiguousarray(l2, dtype=np.int32)
        return int(lib().orc_seed_l2(self._h, _p32(a), int(a.shape[1]), int(tid), int(ts), int(tns)))

    def l2(self, levels=10):
        out = np.zeros((2, levels, 2), np.int32)
        lib().orc_l2(self._h, levels, _p32(out))
        return out

    def dump(self, side):
        out = np.zeros((self.cap, 6), np.int32)
        n = lib().orc_dump(self._h, int(side), _p32(out))
        return out[:n].copy()

    def stats(self):
        s = Stats()
        lib().orc_get_stats(self._h, ctypes.byref(s))
        return {f: getattr(s, f) for f, _ in Stats._fields_ if f != "pad"}


def trade_bound(n_msgs):
    """Trades a book can generate: every trade empties its standing order (at most
    once per resting order, and every resting order came from a limit message) or
    exhausts its aggressor (at most once per message), so trades <= 2 * messages."""
    return 2 * np.asarray(n_msgs, dtype=np.int64)


def default_threads():
    """Worker threads when the caller names none: the cores this process may use,
    at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def run(caps, msgs, offs, l2_mode=L2_NONE, levels=10, trade_room=None, dumps=False,
        dump_cap=None, threads=None):
    """Run every book's stream through the oracle.

    caps[n], msgs[total, 8] int32, offs[n+1] int64.  trade_room[n] = records kept
    per book (default: the bound 2 * messages).  Returns a dict with trades (8-field
    records, concatenated per book), trade_msg (message index of each trade),
    trade_offs, trade_counts, stats, l2, dumps."""
    caps = np.ascontiguousarray(caps, dtype=np.int32)
    msgs = np.ascontiguousarray(msgs, dtype=np.int32).reshape(-1, 8)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    n = caps.shape[0]
    assert offs.shape[0] == n + 1
    if trade_room is None:
        trade_room = trade_bound(np.diff(offs))
    trade_room = np.asarray(trade_room, dtype=np.int64)
    toffs = np.zeros(n + 1, np.int64)
    np.cumsum(trade_room, out=toffs[1:])
    trades = np.full((int(toffs[-1]), 8), -1, np.int32)
    tmsg = np.full(int(toffs[-1]), -1, np.int64)
    counts = np.zeros(n, np.int64)
    stats = np.zeros(n, STATS_DTYPE)
    if l2_mode == L2_PER_MESSAGE:
        l2 = np.zeros((msgs.shape[0], 2, levels, 2), np.int32)
    elif l2_mode == L2_FINAL:
        l2 = np.zeros((n, 2, levels, 2), np.int32)
    else:
        l2 = None
    dcap = int(dump_cap or (caps.max() if n else 1))
    dump_arr = np.zeros((n, 2, dcap, 6), np.int32) if dumps else None
    nt = threads or default_threads()
    rc = lib().orc_run(n, _p32(caps), _p32(msgs), _p64(offs), l2_mode, levels, _p32(l2),
                       _p32(trades), _p64(toffs), _p64(tmsg), _p64(counts), stats.ctypes.data,
                       _p32(dump_arr), dcap, nt)
    if rc != 0:
        raise RuntimeError("orc_run failed")
    kept = np.minimum(counts, trade_room)
    # compact: drop the unused tail of every book's room
    idx = np.concatenate([np.arange(toffs[i], toffs[i] + kept[i]) for i in range(n)]) if n else \
        np.zeros(0, np.int64)
    koffs = np.zeros(n + 1, np.int64)
    np.cumsum(kept, out=koffs[1:])
    return {"trades": trades[idx], "trade_msg": tmsg[idx], "trade_offs": koffs,
            "trade_counts": counts, "stats": stats, "l2": l2, "dumps": dump_arr}
