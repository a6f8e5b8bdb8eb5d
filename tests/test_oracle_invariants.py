"""Oracle against properties the paper and arithmetic fix, on generated order flow,
and against closed forms for special cases.

Properties checked after every message (Section 4.1 / 4.2):
  * the book is never crossed or locked (matching runs while prices overlap,
    inclusively, so no overlap survives a message);
  * shares are conserved: submitted = resting + 2 * traded + cancelled
    + market remainder discarded + rejected;
  * a limit/market message fills exactly a priority-ordered prefix of the
    opposite side, all but the last of them completely (price-time priority),
    at the standing order's price and the aggressor's time, with the aggressor's
    id; no message makes more trades than there were opposite orders.
The priority order used here is the test's own (numpy lexsort on price, time).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2308_13289_amd import workload as W


def ranked(rows, side):
    """rows [n,6] (P,Q,OID,TID,Ts,Tns) sorted into price-time priority."""
    if len(rows) == 0:
        return rows
    price = -rows[:, 0].astype(np.int64) if side == 1 else rows[:, 0].astype(np.int64)
    order = np.lexsort((rows[:, 5], rows[:, 4], price))
    return rows[order]


def live_rows(b, side):
    d = b.dump(side)
    return ranked(d, side)


def check_stream(cap, msgs):
    b = O.Book(cap)
    for m in msgs:
        T, S = int(m[0]), int(m[1])
        before = {s: live_rows(b, s) for s in (1, -1)}
        trades = b.process(m)
        after = {s: live_rows(b, s) for s in (1, -1)}
        st = b.stats()
        # never crossed or locked
        if len(after[1]) and len(after[-1]):
            assert after[1][0, 0] < after[-1][0, 0], (m, after[1][0], after[-1][0])
        # conservation
        resting = int(after[1][:, 1].sum() + after[-1][:, 1].sum()) if True else 0
        assert st["limit_qty"] + st["market_qty"] == (
            resting + 2 * st["traded_qty"] + st["cancelled_qty"] + st["market_discarded"]
            + st["rejected_qty"]), m
        if T in (1, 4):
            opp = before[-S]
            assert len(trades) <= len(opp)
            for k, t in enumerate(trades):
                P, Qt, pas, agg, ts, tns = (int(v) for v in t[:6])
                assert Qt > 0
                # k-th fill is the k-th order in priority, at its own price
                assert pas == opp[k, 2] and P == opp[k, 0], (m, k, t, opp[:k + 1])
                assert agg == m[4] and ts == m[6] and tns == m[7]
                if k < len(trades) - 1:
                    assert Qt == opp[k, 1]  # fully filled before the next is touched
                else:
                    assert Qt <= opp[k, 1]
            if trades.shape[0]:
                lim = m[2] if T == 1 else (2 ** 31 - 1 if S == 1 else 0)
                assert all((t[0] <= lim) if S == 1 else (t[0] >= lim) for t in trades)
        else:
            assert len(trades) == 0
    return b


@pytest.mark.parametrize("book", [0, 1, 2, 3, 17, 42])
def test_invariants_uniform_flow(book):
    w = W.c0()
    check_stream(100, w.msgs[w.offs[book]:w.offs[book + 1]])


def test_invariants_small_capacity_flow():
    """Capacity 8 with 4 seeds per side: sides fill up and reject."""
    w = W.uniform(4, 1500, cap=8, tag=90)
    rejected = 0
    for i in range(4):
        b = check_stream(8, w.msgs[w.offs[i]:w.offs[i + 1]])
        rejected += b.stats()["rejected_qty"]
    assert rejected > 0


def test_invariants_ragged_sample():
    w = W.ragged(n_books=6, max_flow=1500)
    for i in range(w.n_books):
        check_stream(int(w.caps[i]), w.msgs[w.offs[i]:w.offs[i + 1]])


def test_generated_cancels_all_hit():
    """The generator's own ledger (independent code) and the oracle agree on which
    orders are live and how much rests: every generated cancel/delete finds its
    order and removes exactly its quantity; nothing is rejected at capacity 100."""
    w = W.uniform(64, 3000, tag=91)
    r = O.run(w.caps, w.msgs, w.offs)
    st = r["stats"]
    assert st["cancel_miss"].sum() == 0
    assert st["rejected_qty"].sum() == 0
    for i in range(w.n_books):
        m = w.msgs[w.offs[i]:w.offs[i + 1]]
        cq = m[(m[:, 0] == 2) | (m[:, 0] == 3), 3].astype(np.int64).sum()
        assert st["cancelled_qty"][i] == cq


def test_trade_bound_and_l2_groupby():
    """trades <= 2 * messages per book; final L2 = group-by-price of the final book
    (numpy unique + bincount)."""
    w = W.uniform(32, 2000, tag=92)
    r = O.run(w.caps, w.msgs, w.offs, l2_mode=O.L2_FINAL, levels=10, dumps=True)
    n = np.diff(w.offs)
    assert (r["trade_counts"] <= 2 * n).all()
    for i in range(w.n_books):
        for sd, side in ((0, -1), (1, 1)):
            d = r["dumps"][i, sd]
            d = d[d[:, 1] > 0]
            prices, inv = np.unique(d[:, 0], return_inverse=True)
            sums = np.bincount(inv, weights=d[:, 1]).astype(np.int64)
            if side == 1:
                prices, sums = prices[::-1], sums[::-1]
            want = np.full((10, 2), [-1, 0], np.int64)
            k = min(10, len(prices))
            want[:k, 0], want[:k, 1] = prices[:k], sums[:k]
            np.testing.assert_array_equal(r["l2"][i, sd], want)


@pytest.mark.parametrize("seed", range(5))
def test_single_level_is_fifo(seed):
    """One price, no cancels: the book is a FIFO queue.  The fills are the
    overlaps of the resting orders' cumulative-quantity intervals with the market
    orders' cumulative-quantity intervals."""
    rng = np.random.default_rng(seed)
    rest = rng.integers(1, 50, size=30)
    mkt = rng.integers(1, 80, size=25)
    msgs = [[1, -1, 500, int(q), i + 1, 7, 34200, i] for i, q in enumerate(rest)]
    base = len(rest)
    msgs += [[4, 1, 0, int(q), 1000 + j, 8, 34201, j] for j, q in enumerate(mkt)]
    b = O.Book(64)
    got = []
    for k, m in enumerate(msgs):
        for t in b.process(m):
            got.append((k - base, int(t[2]) - 1, int(t[1])))
    R = np.concatenate([[0], np.cumsum(rest)])
    M = np.concatenate([[0], np.cumsum(mkt)])
    want = []
    for j in range(len(mkt)):
        lo, hi = M[j], min(M[j + 1], R[-1])
        for i in range(len(rest)):
            a, c = max(lo, R[i]), min(hi, R[i + 1])
            if c > a:
                want.append((j, i, int(c - a)))
    assert got == want


@pytest.mark.parametrize("seed", range(5))
def test_market_walks_static_book(seed):
    """A market order against a static multi-level book fills min(Q, depth), and
    its notional is the closed-form walk: sum_l P_l * clip(Q - C_{l-1}, 0, q_l)."""
    rng = np.random.default_rng(100 + seed)
    prices = rng.choice(np.arange(990, 1010), size=12, replace=True)
    qtys = rng.integers(1, 40, size=12)
    msgs = [[1, -1, int(p), int(q), i + 1, 7, 34200, i] for i, (p, q) in enumerate(zip(prices, qtys))]
    Q = int(rng.integers(1, qtys.sum() + 30))
    b = O.Book(16)
    for m in msgs:
        b.process(m)
    tr = b.process([4, 1, 0, Q, 999, 8, 34201, 0])
    lv_p, inv = np.unique(prices, return_inverse=True)
    lv_q = np.bincount(inv, weights=qtys).astype(np.int64)
    C = np.concatenate([[0], np.cumsum(lv_q)])
    take = np.clip(Q - C[:-1], 0, lv_q)
    assert tr[:, 1].sum() == min(Q, qtys.sum())
    assert (tr[:, 0].astype(np.int64) * tr[:, 1]).sum() == (lv_p * take).sum()
    assert b.stats()["market_discarded"] == max(0, Q - int(qtys.sum()))


def test_time_order_flag():
    b = O.Book(4)
    b.process([1, 1, 100, 1, 1, 0, 34200, 5])
    b.process([1, 1, 100, 1, 2, 0, 34200, 5])  # equal time: allowed
    assert b.stats()["flags"] & O.FLAG_TIME_ORDER == 0
    b.process([1, 1, 100, 1, 3, 0, 34200, 4])
    assert b.stats()["flags"] & O.FLAG_TIME_ORDER
