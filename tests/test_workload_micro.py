"""Inputs of the operation microbenchmark (paper Tables 1-4) do what they claim,
checked with the oracle: the seeds fill one third of each side without crossing,
adds rest without trading, cancels hit resting orders, crossing limits and market
orders trade."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2308_13289_amd import workload as W


def replay(N, seeds, msg):
    o = O.run(np.array([N], np.int32), np.concatenate([seeds, msg]), np.array([0, len(seeds) + 1], np.int64),
              dumps=True, dump_cap=N)
    return o


@pytest.mark.parametrize("N", [10, 100, 1000])
def test_seeds_fill_one_third_without_crossing(N):
    seeds, rest = W.micro_book(N)
    n = max(1, N // 3)
    assert len(seeds) == 2 * n
    asks, bids = seeds[seeds[:, 1] == -1], seeds[seeds[:, 1] == 1]
    assert len(asks) == len(bids) == n
    assert asks[:, 2].min() > W.MICRO_MID > bids[:, 2].max()
    o = O.run(np.array([N], np.int32), seeds, np.array([0, len(seeds)], np.int64), dumps=True, dump_cap=N)
    assert o["trade_counts"][0] == 0
    d = o["dumps"][0]
    assert (d[0, :, 3] > 0).sum() == n and (d[1, :, 3] > 0).sum() == n


@pytest.mark.parametrize("N", [10, 100, 1000])
def test_ops_behave_as_named(N):
    seeds, rest = W.micro_book(N)
    n = max(1, N // 3)
    for m in W.micro_messages(N, "add", 20):
        o = replay(N, seeds, m[None])
        assert o["trade_counts"][0] == 0
        assert (o["dumps"][0][:, :, 3] > 0).sum() == 2 * n + 1
    live = {int(r[3]): int(r[2]) for r in rest}
    for m in W.micro_messages(N, "cancel", 20):
        assert m[4] in live and 1 <= m[3] <= live[m[4]]
        o = replay(N, seeds, m[None])
        assert o["trade_counts"][0] == 0 and o["stats"]["cancel_miss"][0] == 0
        assert o["stats"]["cancelled_qty"][0] == m[3]
    for m in W.micro_messages(N, "match", 20):
        o = replay(N, seeds, m[None])
        assert o["trade_counts"][0] >= 1


def test_market_sizes():
    seeds, rest = W.micro_book(100)
    for q in (0, 10, 500, 1000, 10000):
        m = W.micro_messages(100, "market", 5, market_qty=q)
        assert (m[:, 0] == 4).all() and (m[:, 3] == q).all()
        for k in range(len(m)):
            o = replay(100, seeds, m[k:k + 1])
            # a market order trades min(q, everything resting on the opposite side)
            opposite = rest[rest[:, 0] == -m[k, 1], 2].sum()
            assert o["stats"]["traded_qty"][0] == min(q, opposite)
            assert (o["trade_counts"][0] == 0) == (q == 0)
