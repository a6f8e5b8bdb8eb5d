"""Execution-environment oracle (JAX-LOB Section 5.2; readings R15-R18 in
oracle/exec_env.py), pinned by hand-worked steps: the observation fields, the
VWAP reward of eqs. (rewardfunc) and (vwap), the forced market order one minute
before the end, and the cap of the executed quantity at the task size."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle.exec_env import ExecEnv

AGENT = -1


def book_with(asks, bids):
    """asks / bids: (price, qty) resting orders placed at time (1, k) by trader 5."""
    b = O.Book(16)
    oid = 1
    for k, (p, q) in enumerate(asks):
        b.process([1, -1, p, q, oid, 5, 1, k])
        oid += 1
    for k, (p, q) in enumerate(bids):
        b.process([1, 1, p, q, oid, 5, 1, 100 + k])
        oid += 1
    return b


def test_hand_worked_sell_step():
    # asks 101 x 5, 102 x 5; bids 99 x 5.  A data buyer takes 3 @ 101; the agent
    # (sell task of 10, action: 2 at the far touch = best bid 99) sells 2 @ 99.
    b = book_with([(101, 5), (102, 5)], [(99, 5)])
    env = ExecEnv(b, task_side=-1, task_qty=10, p_init=100, start=(2, 0), end_s=1000, next_oid=7000,
                  tick=1, passive_ticks=1, agent_tid=AGENT, lam=0.5)
    window = np.array([[1, 1, 102, 3, 50, 6, 3, 500]], np.int32)
    obs, reward, fills = env.step(window, [2, 0, 0, 0])
    # trades: (101, 3) data, (99, 2) agent: VWAP = (303 + 198) / 5 = 100.2
    # R = 2 (99 - 100.2) + 0.5 * 2 (100.2 - 100) = -2.4 + 0.2
    assert reward == pytest.approx(-2.2, abs=1e-12)
    np.testing.assert_array_equal(fills, [[99, 2, 3, 7000, 3, 500]])
    W = 1
    # after the data message: ask 101 x 2, bid 99 x 5
    assert obs[0] == 99 and obs[W] == 101 and obs[2 * W] == 100  # bid, ask, mid
    assert obs[3 * W] == 102                                     # passive: ask + 1 tick (sell task)
    assert obs[4 * W] == 2 and obs[5 * W] == 2 - 5               # spread, imbalance
    np.testing.assert_array_equal(obs[6 * W:], [3, 500, 1, 500, 100, 0, 10, 2])
    assert env.exec_qty == 2 and env.revenue == 198 and env.next_oid == 7001 and env.done == 0


def test_prices_of_the_four_action_levels_buy():
    # buy task: far touch = ask 110, mid = floor((110 + 97) / 2) = 103, near = bid 97,
    # passive = 97 - 2 ticks of 1
    b = book_with([(110, 50)], [(97, 50)])
    env = ExecEnv(b, task_side=1, task_qty=100, p_init=103, start=(2, 0), end_s=1000, next_oid=1,
                  tick=1, passive_ticks=2, agent_tid=AGENT)
    env.step(np.array([[0] * 8], np.int32), [1, 2, 3, 4])
    asks, bids = b.dump(0), b.dump(1)
    # the far-touch buy of 1 traded with the ask; the others rest at 103, 97, 95
    assert asks[0, 1] == 49
    got = {int(r[0]): int(r[1]) for r in bids if r[3] == AGENT}
    assert got == {103: 2, 97: 3, 95: 4}


def test_forced_market_order_and_done():
    b = book_with([(101, 4), (103, 10)], [(99, 5)])
    env = ExecEnv(b, task_side=1, task_qty=9, p_init=100, start=(2, 0), end_s=62, next_oid=1, tick=1,
                  agent_tid=AGENT)
    # the data message time 2 s >= end_s - 60: the action is ignored, a market buy of 9 goes in
    obs, reward, fills = env.step(np.array([[2, 1, 99, 1, 3, 5, 2, 0]], np.int32), [1, 1, 1, 1])
    np.testing.assert_array_equal(fills[:, :2], [[101, 4], [103, 5]])
    assert env.exec_qty == 9 and env.done == 1 and env.next_oid == 2
    # all trades are the agent's: P_VWAP equals its own average, the advantage is 0
    assert reward == pytest.approx(0.0, abs=1e-12)
    # a done task sends nothing
    env.step(np.array([[0] * 8], np.int32), [5, 5, 5, 5])
    assert env.next_oid == 2


def test_executed_quantity_capped_at_task():
    b = book_with([(101, 50)], [(99, 5)])
    env = ExecEnv(b, task_side=1, task_qty=3, p_init=100, start=(2, 0), end_s=1000, next_oid=1, tick=1,
                  agent_tid=AGENT, lam=1.0)
    obs, reward, fills = env.step(np.array([[0] * 8], np.int32), [8, 0, 0, 0])
    assert fills[0, 1] == 8 and env.exec_qty == 3 and env.revenue == 303
    # VWAP 101 (the only trade): R = 3 (101 - 101) + 1 * 3 (101 - 100) = 3
    assert reward == pytest.approx(3.0, abs=1e-12)
    assert obs[-1] == 3 and env.done == 1
