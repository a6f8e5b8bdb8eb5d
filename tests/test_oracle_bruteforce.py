"""Brute force on tiny books: every message sequence of a small alphabet, run
through the oracle and through the independent naive engine, must give the same
trades, per-message L2, final books and counters.

The alphabet covers every message type and side, prices that do and do not
cross, quantities below / equal to / above the resting ones, cancels of live,
filled, unknown and initial (Section 5.1.1) orders, and capacities small enough
that a side fills up.
"""
import itertools

import numpy as np
import pytest

from naive_engine import NaiveBook
from oracle import oracle as O

# two initial orders (Section 5.1.1 ids), one per side
PREFIX = [[1, -1, 3, 2, -9000, 0, 34199, 0], [1, 1, 1, 2, -9001, 0, 34199, 1]]
LEVELS = 2


def alphabet():
    items = []
    for S in (1, -1):
        for P in (1, 2, 3):
            for Q in (1, 2, 3):
                items.append((1, S, P, Q, None))
        for Q in (1, 3):
            items.append((4, S, 2, Q, None))
        for tgt in (1, 2):
            for Q in (1, 2):
                items.append((2, S, 2, Q, tgt))
        for P in (1, 3):
            for Q in (1, 2):
                items.append((2, S, P, Q, 77))
        items.append((3, S, 2, 3, 1))
        items.append((3, S, 3, 3, 77))
    return items


def to_msgs(seq, prefix=PREFIX, times=None):
    """Messages of one sequence after the prefix; message k is stamped (34200, k),
    or (34200, times[k]) when times are given (equal and decreasing times)."""
    msgs = [list(m) for m in prefix]
    for k, (T, S, P, Q, tgt) in enumerate(seq):
        oid = k + 1 if tgt is None else tgt
        msgs.append([T, S, P, Q, oid, 10 + k % 3, 34200, k if times is None else int(times[k])])
    return msgs


BIG = 2 ** 31 - 1
# initial orders of the large-quantity runs: INT32_MAX shares each
PREFIX_BIG = [[1, -1, 3, BIG, -9000, 0, 34199, 0], [1, 1, 1, BIG, -9001, 0, 34199, 1]]


def alphabet_big():
    """Quantities near 2^31 (Section 4.2: Q is an int32 field): sweeps whose fills
    add up past INT32_MAX, cancels larger than the resting quantity, L2 levels whose
    sums pass INT32_MAX."""
    items = []
    for S in (1, -1):
        for P in (1, 2, 3):
            for Q in (1, 1_500_000_000, BIG):
                items.append((1, S, P, Q, None))
        for Q in (2_100_000_000, BIG):
            items.append((4, S, 2, Q, None))
        for tgt in (1, 2):
            items.append((2, S, 2, 2_000_000_000, tgt))
            items.append((2, S, 2, 1, tgt))
        items.append((3, S, 3, BIG, 1))
    return items


def compare(seqs, cap, prefix=PREFIX, times=None):
    streams = [to_msgs(s, prefix, None if times is None else times[i]) for i, s in enumerate(seqs)]
    lens = [len(s) for s in streams]
    offs = np.zeros(len(streams) + 1, np.int64)
    np.cumsum(lens, out=offs[1:])
    msgs = np.array([m for s in streams for m in s], np.int32)
    r = O.run(np.full(len(streams), cap), msgs, offs, l2_mode=O.L2_PER_MESSAGE, levels=LEVELS,
              dumps=True, dump_cap=cap)
    for i, stream in enumerate(streams):
        nb = NaiveBook(cap)
        trades, l2s = [], []
        for m in stream:
            trades.extend(nb.process(m))
            l2s.append(nb.l2(LEVELS))
        got_tr = r["trades"][r["trade_offs"][i]:r["trade_offs"][i + 1]]
        ctx = f"cap={cap} seq={seqs[i]}"
        assert got_tr.tolist() == trades, ctx
        assert r["l2"][offs[i]:offs[i + 1]].tolist() == l2s, ctx
        for sd, side in ((0, -1), (1, 1)):
            want = nb.dump(side)
            got = r["dumps"][i][sd]
            assert got[:len(want)].tolist() == want, ctx
            assert (got[len(want):] == -1).all(), ctx
        st = r["stats"][i]
        assert (st["rejected_qty"], st["cancelled_qty"], st["market_discarded"],
                st["cancel_miss"]) == (nb.rejected, nb.cancelled, nb.discarded, nb.misses), ctx


@pytest.mark.parametrize("cap", [1, 2])
def test_exhaustive_length3(cap):
    A = alphabet()
    compare(list(itertools.product(A, repeat=3)), cap)


@pytest.mark.parametrize("cap,length", [(2, 8), (3, 12)])
def test_random_sequences(cap, length):
    A = alphabet()
    rng = np.random.default_rng(1000 * cap + length)
    seqs = [[A[j] for j in rng.integers(0, len(A), size=length)] for _ in range(6000)]
    compare(seqs, cap)


@pytest.mark.parametrize("cap", [2, 3])
def test_exhaustive_length3_large_quantities(cap):
    compare(list(itertools.product(alphabet_big(), repeat=3)), cap, prefix=PREFIX_BIG)


def test_random_sequences_large_quantities():
    A = alphabet_big()
    rng = np.random.default_rng(77)
    seqs = [[A[j] for j in rng.integers(0, len(A), size=10)] for _ in range(6000)]
    compare(seqs, 4, prefix=PREFIX_BIG)


@pytest.mark.parametrize("cap", [2, 3])
def test_random_sequences_times_out_of_order(cap):
    """Times drawn from a few values, so that equal and decreasing times occur: the
    priority among equal prices follows the time stamps (Section 4.1), then arrival."""
    A = alphabet()
    rng = np.random.default_rng(500 + cap)
    seqs = [[A[j] for j in rng.integers(0, len(A), size=10)] for _ in range(6000)]
    times = rng.integers(0, 4, size=(len(seqs), 10))
    compare(seqs, cap, times=times)
