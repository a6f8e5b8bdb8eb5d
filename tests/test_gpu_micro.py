"""The single-message calls of the operation microbenchmark (a book of capacity N
filled to one third per side; add / cancel / match / market messages): for one
book and for several identical books, trades and the book after each call equal
the oracle's (tolerance 0: everything is integer)."""
import numpy as np
import pytest
import torch

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_helpers import to_dev  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2308_13289_amd import lob  # noqa: E402
from paper_2308_13289_amd import workload as W  # noqa: E402

CASES = [(N, op, None) for N in (10, 100, 1000) for op in W.MICRO_OPS] + \
        [(100, "market", q) for q in (0, 10, 500, 1000, 10000)]
RESIDENCY = {"regs": {"registers": 1}, "lds": {"registers": 0}, "unsorted": {"layout": 1}}


def oracle_after(N, seeds, msg):
    o = O.run(np.array([N], np.int32), np.concatenate([seeds, msg]), np.array([0, len(seeds) + 1], np.int64),
              dumps=True, dump_cap=N)
    return o["trades"][:, :6], o["dumps"][0]


@pytest.mark.parametrize("res", list(RESIDENCY))
@pytest.mark.parametrize("N,op,q", CASES)
def test_micro_calls_match_oracle(N, op, q, res):
    n_books, trials = 3, 6
    seeds, _ = W.micro_book(N)
    msgs = W.micro_messages(N, op, trials, market_qty=q)
    ctx = lob.Context(np.full(n_books, N, np.int32), l2_levels=10, trade_log_records=2 * N + 64)
    ctx.set_plan(**RESIDENCY[res])
    ctx.process(to_dev(np.tile(seeds, (n_books, 1))), to_dev(np.arange(n_books + 1, dtype=np.int64) * len(seeds)))
    dump = ctx.read_book(N)
    one = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    for t in range(trials):
        want_tr, want_book = oracle_after(N, seeds, msgs[t:t + 1])
        # one book
        ctx.reset(book_ids=one)
        ctx.write_book(dump[:1], book_ids=one)
        ctx.process(to_dev(msgs[t:t + 1]), to_dev(np.array([0, 1], np.int64)), book_ids=one)
        total = int(ctx.read_status(one)["log_records"].sum())
        rec, _, _ = ctx.read_trades(max(total, 1), book_ids=one)
        np.testing.assert_array_equal(rec[:total].cpu().numpy(), want_tr, err_msg=f"trial {t}")
        np.testing.assert_array_equal(ctx.read_book(N, book_ids=one)[0].cpu().numpy(), want_book)
        # the same message to every book
        ctx.reset()
        ctx.write_book(dump)
        ctx.process(to_dev(np.repeat(msgs[t:t + 1], n_books, axis=0)), to_dev(np.arange(n_books + 1, dtype=np.int64)))
        st = ctx.read_status()
        assert (st["log_records"] == len(want_tr)).all()
        books = ctx.read_book(N).cpu().numpy()
        for b in range(n_books):
            np.testing.assert_array_equal(books[b], want_book)
    ctx.close()
