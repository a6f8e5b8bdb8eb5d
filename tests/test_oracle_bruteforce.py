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


def to_msgs(seq):
    msgs = [list(m) for m in PREFIX]
    for k, (T, S, P, Q, tgt) in enumerate(seq):
        oid = k + 1 if tgt is None else tgt
        msgs.append([T, S, P, Q, oid, 10 + k % 3, 34200, k])
    return msgs


def compare(seqs, cap):
    streams = [to_msgs(s) for s in seqs]
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
