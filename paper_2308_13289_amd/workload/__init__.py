"""Seeded synthetic order-flow workloads (binding of flowgen.c).

The workloads stand in for the paper's LOBSTER message data (JAX-LOB, Section 5:
TSLA 2015-01-02 and AMZN April 2021), which is not available here: same message
structure, prices on a tick grid around a mid price, LOBSTER-like mix of limit,
cancel, delete and market messages, strictly increasing times.

  uniform(...)   books of one capacity, same flow length      (64 x 1000; 4096 x 10000)
  ragged(...)    capacity in {50,100,500,1000}, log-uniform flow length 1e2..1e5
  step_windows   100-message windows plus agent actions for the env-step form
"""
import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "flowgen.c")
LIB = os.path.join(HERE, "libflowgen.so")

SEED = 230813289
TICK = 100
TAGS = {"c0": 0, "c1": 1, "c2": 2, "c3": 3, "c4": 4}


def build(force=False):
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "flowgen.h"))):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                           "-pthread", SRC, "-lm", "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        vp, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, \
            ctypes.c_uint64
        L.fg_generate.restype = i32
        L.fg_generate.argtypes = [u64, u32, i32, vp, vp, i32, vp, vp, vp, vp, vp, i32]
        L.fg_agent.restype = i32
        L.fg_agent.argtypes = [u64, u32, i32, vp, vp, i32, i32, vp, vp, i32]
        L.fg_ragged_params.restype = None
        L.fg_ragged_params.argtypes = [u64, u32, i32, vp, vp, vp]
        L.fg_requests.restype = None
        L.fg_requests.argtypes = [u64, u32, i64, ctypes.c_double, i32, vp, vp, vp, vp]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _threads(threads):
    return int(threads or min(os.cpu_count() or 1, 16))


@dataclass
class Workload:
    """Message streams of a batch of books: book i reads msgs[offs[i]:offs[i+1]]."""
    name: str
    caps: np.ndarray          # int32 [n]     capacity per side
    mids: np.ndarray          # int32 [n]
    seeds_per_side: np.ndarray  # int32 [n]
    n_flow: np.ndarray        # int64 [n]     flow messages after the seed block
    msgs: np.ndarray          # int32 [total, 8]
    offs: np.ndarray          # int64 [n + 1]
    extra: dict = field(default_factory=dict)

    @property
    def n_books(self):
        return int(self.caps.shape[0])

    @property
    def n_msgs(self):
        return int(self.offs[-1])


def generate(tag, caps, mids, seeds_per_side, n_flow, key_ids=None, seed=SEED, tick=TICK,
             threads=None, name=None):
    caps = np.ascontiguousarray(caps, np.int32)
    mids = np.ascontiguousarray(mids, np.int32)
    spb = np.ascontiguousarray(seeds_per_side, np.int32)
    n_flow = np.ascontiguousarray(n_flow, np.int64)
    n = caps.shape[0]
    lens = 2 * spb.astype(np.int64) + n_flow
    offs = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=offs[1:])
    msgs = np.empty((int(offs[-1]), 8), np.int32)
    kid = None if key_ids is None else np.ascontiguousarray(key_ids, np.int32)
    rc = lib().fg_generate(seed, tag, n, _ptr(kid), _ptr(mids), tick, _ptr(caps), _ptr(spb),
                           _ptr(n_flow), _ptr(msgs), _ptr(offs), _threads(threads))
    if rc != 0:
        raise ValueError("fg_generate: bad arguments")
    return Workload(name or f"tag{tag}", caps, mids, spb, n_flow, msgs, offs)


def uniform(n_books, n_flow, cap=100, mid=10_000_000, tag=TAGS["c0"], seed=SEED, threads=None,
            name=None):
    """Books of one capacity, seeded with cap/2 orders per side, n_flow messages each."""
    return generate(tag, np.full(n_books, cap), np.full(n_books, mid), np.full(n_books, cap // 2),
                    np.full(n_books, n_flow), seed=seed, threads=threads,
                    name=name or f"uniform{n_books}x{n_flow}c{cap}")


def c0(**kw):
    """64 books, capacity 100, 1000 flow messages per book."""
    return uniform(64, 1000, tag=TAGS["c0"], name="c0_64x1000_cap100", **kw)


def c1(**kw):
    """4096 books, capacity 100, 10000 flow messages per book."""
    return uniform(4096, 10_000, tag=TAGS["c1"], name="c1_4096x10000_cap100", **kw)


def ragged_params(n_books, seed=SEED, tag=TAGS["c2"]):
    caps = np.empty(n_books, np.int32)
    n_flow = np.empty(n_books, np.int64)
    mids = np.empty(n_books, np.int32)
    lib().fg_ragged_params(seed, tag, n_books, _ptr(caps), _ptr(n_flow), _ptr(mids))
    return caps, n_flow, mids


def ragged(n_books=10_000, seed=SEED, tag=TAGS["c2"], threads=None, max_flow=None):
    """Mixed capacities {50,100,500,1000}, flow length log-uniform in [1e2, 1e5].
    max_flow (tests only) caps the flow length to keep a case small."""
    caps, n_flow, mids = ragged_params(n_books, seed, tag)
    if max_flow is not None:
        n_flow = np.minimum(n_flow, max_flow)
    return generate(tag, caps, mids, caps // 2, n_flow, seed=seed, threads=threads,
                    name=f"ragged{n_books}")


def agent_actions(tag, mids, n_steps, times, key_ids=None, seed=SEED, tick=TICK, threads=None):
    """[n][steps][4][8] agent orders; times[n][steps][2] = time of each step's last
    data message."""
    mids = np.ascontiguousarray(mids, np.int32)
    times = np.ascontiguousarray(times, np.int32)
    n = mids.shape[0]
    out = np.empty((n, n_steps, 4, 8), np.int32)
    kid = None if key_ids is None else np.ascontiguousarray(key_ids, np.int32)
    rc = lib().fg_agent(seed, tag, n, _ptr(kid), _ptr(mids), tick, n_steps, _ptr(times), _ptr(out),
                        _threads(threads))
    if rc != 0:
        raise ValueError("fg_agent: bad arguments")
    return out


def step_workload(n_books=8192, n_steps=1000, window=100, cap=100, mid=10_000_000,
                  tag=TAGS["c3"], seed=SEED, threads=None):
    """Environment-step form: each book is seeded (cap/2 orders per side), then every
    step replays `window` data messages and then up to 4 agent orders.
    Returns the Workload of the data streams (seed block + n_steps*window flow) and
    puts `actions` [n][steps][4][8] into .extra."""
    w = uniform(n_books, n_steps * window, cap=cap, mid=mid, tag=tag, seed=seed, threads=threads,
                name=f"step{n_books}x{n_steps}x{window}")
    seeds = 2 * (cap // 2)
    flow = w.msgs.reshape(n_books, seeds + n_steps * window, 8)[:, seeds:, :]
    last = flow.reshape(n_books, n_steps, window, 8)[:, :, window - 1, 6:8]
    w.extra["actions"] = agent_actions(tag, w.mids, n_steps, last, seed=seed, threads=threads)
    w.extra["window"] = window
    w.extra["n_steps"] = n_steps
    w.extra["seed_msgs"] = seeds
    return w


def requests(n_req, lam, n_books, seed=SEED, tag=TAGS["c4"]):
    arr = np.empty(n_req, np.int64)
    book = np.empty(n_req, np.int32)
    kind = np.empty(n_req, np.int32)
    size = np.empty(n_req, np.int32)
    lib().fg_requests(seed, tag, n_req, float(lam), n_books, _ptr(arr), _ptr(book), _ptr(kind),
                      _ptr(size))
    return arr, book, kind, size


# ---------------------------------------------------------------- operation microbenchmarks
# Inputs for the paper's per-operation timings (Section 4.1, Tables 1-4): a book of
# capacity N filled to one third per side with random orders, and single messages
# that add without crossing, cancel a resting order, cross the spread, or are market
# orders of a given size.

MICRO_OPS = ("add", "cancel", "match")
MICRO_MID = 10_000_000


def _micro_rng(cap, what, seed):
    return np.random.Generator(np.random.PCG64([seed, 0x51C0, int(cap), int(what)]))


def _qty(rng, n):
    return np.minimum(1 + np.floor(rng.lognormal(4.0, 1.0, n)), 10_000).astype(np.int32)


def micro_book(cap, seed=SEED, mid=MICRO_MID, tick=TICK):
    """Seed messages filling a book of capacity `cap` to one third per side (at least
    one order each): limit asks at mid + k*tick and bids at mid - k*tick with
    k = 1 + Geometric(0.3), qty = 1 + floor(LogNormal(4, 1)) clipped to 10,000, order
    ids 1, 2, ..., times (34199, i).  Returns [2*n][8] int32 and the per-order
    (side, price, qty, oid) table of what rests after them."""
    rng = _micro_rng(cap, 0, seed)
    n = max(1, cap // 3)
    k = rng.geometric(0.3, 2 * n)  # numpy's geometric counts trials: 1 + failures, >= 1
    side = np.repeat(np.array([-1, 1], np.int32), n)
    price = np.where(side == -1, mid + k * tick, mid - k * tick).astype(np.int32)
    qty = _qty(rng, 2 * n)
    oid = np.arange(1, 2 * n + 1, dtype=np.int32)
    m = np.zeros((2 * n, 8), np.int32)
    m[:, 0] = 1
    m[:, 1] = side
    m[:, 2] = price
    m[:, 3] = qty
    m[:, 4] = oid
    m[:, 5] = 7
    m[:, 6] = 34199
    m[:, 7] = np.arange(2 * n, dtype=np.int32)
    return m, np.stack([side, price, qty, oid], axis=1)


def micro_messages(cap, op, n_trials, seed=SEED, mid=MICRO_MID, tick=TICK, market_qty=None):
    """One message per trial, each applied to the freshly restored micro_book:
      add     limit at mid -/+ tick*U{0..5} (buy/sell), never crossing the spread
      cancel  partial-or-full cancel (qty ~ U[1, resting]) of a uniform resting order
      match   limit crossing the spread: buy at mid + 1000*tick / sell at mid - 1000*tick
      market  market order of quantity market_qty (side uniform)
    Returns [n_trials][8] int32 with time (34200, trial)."""
    what = {"add": 1, "cancel": 2, "match": 3, "market": 4}[op]
    rng = _micro_rng(cap, 16 * what + (0 if market_qty is None else 1 + int(market_qty) % 7919), seed)
    _, rest = micro_book(cap, seed=seed, mid=mid, tick=tick)
    t = np.arange(n_trials)
    m = np.zeros((n_trials, 8), np.int32)
    side = np.where(rng.random(n_trials) < 0.5, 1, -1).astype(np.int32)
    m[:, 4] = 1_000_000 + t
    m[:, 5] = 8
    m[:, 6] = 34200
    m[:, 7] = t
    if op == "add":
        off = tick * rng.integers(0, 6, n_trials)
        m[:, 0], m[:, 1] = 1, side
        m[:, 2] = np.where(side == 1, mid - off, mid + off)
        m[:, 3] = _qty(rng, n_trials)
    elif op == "cancel":
        pick = rest[rng.integers(0, rest.shape[0], n_trials)]
        m[:, 0], m[:, 1], m[:, 2] = 2, pick[:, 0], pick[:, 1]
        m[:, 3] = 1 + np.floor(rng.random(n_trials) * pick[:, 2]).astype(np.int32)
        m[:, 4] = pick[:, 3]
    elif op == "match":
        m[:, 0], m[:, 1] = 1, side
        m[:, 2] = np.where(side == 1, mid + 1000 * tick, mid - 1000 * tick)
        m[:, 3] = _qty(rng, n_trials)
    elif op == "market":
        m[:, 0], m[:, 1] = 4, side
        m[:, 2] = 0
        m[:, 3] = int(market_qty)
    return m
