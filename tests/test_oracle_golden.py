"""Oracle against the hand-worked cases of tests/golden (each cites the paper)."""
import numpy as np
import pytest

from golden_cases import all_cases
from oracle import oracle as O

CASES = all_cases()


@pytest.mark.parametrize("case", CASES, ids=[c.name for c in CASES])
def test_golden_case(case):
    b = O.Book(case.cap)
    got = []
    for k, m in enumerate(case.msgs):
        for t in b.process(m):
            got.append([k] + list(t[:6]))
    got = np.array(got, np.int64).reshape(-1, 7)
    np.testing.assert_array_equal(got, case.trades, err_msg=f"trades ({case.cite})")
    np.testing.assert_array_equal(b.dump(-1), case.ask, err_msg=f"asks ({case.cite})")
    np.testing.assert_array_equal(b.dump(1), case.bid, err_msg=f"bids ({case.cite})")
    l2 = b.l2(case.levels)
    if case.l2ask is not None:
        np.testing.assert_array_equal(l2[0], case.l2ask)
    if case.l2bid is not None:
        np.testing.assert_array_equal(l2[1], case.l2bid)
    st = b.stats()
    for k, v in case.stats.items():
        assert st[k] == v, (k, st[k], v, case.cite)


def test_golden_batch_runner_agrees_with_stepper():
    """orc_run (threads, per-message L2, dumps) gives what the single-book stepper gives."""
    caps = [c.cap for c in CASES]
    msgs = np.concatenate([c.msgs for c in CASES])
    offs = np.concatenate([[0], np.cumsum([len(c.msgs) for c in CASES])]).astype(np.int64)
    r = O.run(caps, msgs, offs, l2_mode=O.L2_PER_MESSAGE, levels=3, dumps=True, threads=4)
    for i, c in enumerate(CASES):
        tr = r["trades"][r["trade_offs"][i]:r["trade_offs"][i + 1], :6]
        np.testing.assert_array_equal(tr, c.trades[:, 1:].astype(np.int32))
        d = r["dumps"][i]
        np.testing.assert_array_equal(d[0][:len(c.ask)], c.ask)
        np.testing.assert_array_equal(d[1][:len(c.bid)], c.bid)
        assert (d[0][len(c.ask):] == -1).all() and (d[1][len(c.bid):] == -1).all()
        last = r["l2"][offs[i + 1] - 1]
        if c.l2ask is not None:
            np.testing.assert_array_equal(last[0], c.l2ask)
        if c.l2bid is not None:
            np.testing.assert_array_equal(last[1], c.l2bid)
