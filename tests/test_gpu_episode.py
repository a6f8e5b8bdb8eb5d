"""An episode the way JAX-LOB's base environment runs one (Section 5.1.1): replay a
book's stream up to a window start, take its L2 snapshot, start a fresh book from
the snapshot (lob_seed_l2), then step through the window's fixed-size steps
(lob_windows + lob_step).  L2 after every step, agent fills and the final book
equal the oracle doing the same (tolerance 0: all integer).  Also the seeding
kernel alone against the oracle's, valid and invalid snapshots."""
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

LEVELS = 10


def oracle_seeded(cap, l2, ts, tns, tid):
    b = O.Book(cap)
    assert b.seed_l2(l2, tid=tid, ts=ts, tns=tns) >= 0
    return b


def test_seed_kernel_matches_oracle():
    rng = np.random.default_rng(5)
    n, cap, L = 64, 12, 10
    snaps = np.zeros((n, 2, L, 2), np.int32)
    snaps[:, :, :, 0] = -1
    for i in range(n):
        na, nb = rng.integers(0, L + 1, 2)
        mid = 10_000 + 100 * int(rng.integers(-50, 50))
        asks = mid + 100 * np.cumsum(rng.integers(1, 4, na))
        bids = mid - 100 * np.cumsum(rng.integers(1, 4, nb))
        snaps[i, 0, :na] = np.stack([asks, rng.integers(1, 500, na)], 1)
        snaps[i, 1, :nb] = np.stack([bids, rng.integers(1, 500, nb)], 1)
        if i % 7 == 0 and na and nb:
            snaps[i, 1, 0, 0] = snaps[i, 0, 0, 0]  # locked: best bid == best ask
        if i % 11 == 3 and na > 1:
            snaps[i, 0, [0, 1]] = snaps[i, 0, [1, 0]]  # unordered
        if i % 13 == 5:
            snaps[i, :, 2, 1] = 0  # a missing level in the middle
    caps = np.full(n, cap, np.int32)
    caps[::9] = 3  # some books too small for their snapshot
    ctx = lob.Context(caps, l2_levels=L, trade_log_records=16)
    times = np.stack([np.full(n, 34500), np.arange(n)], 1).astype(np.int32)
    ctx.seed_l2(to_dev(snaps), times=to_dev(times), init_tid=3)
    dump = ctx.read_book(cap).cpu().numpy()
    st = ctx.read_status()
    flags = st["flags"]
    for i in range(n):
        b = O.Book(int(caps[i]))
        r = b.seed_l2(snaps[i], tid=3, ts=34500, tns=i)
        if r < 0:
            assert flags[i] & lob.BOOK_BAD_LOAD, i
            assert (dump[i][:, :, 1] <= 0).all()
            continue
        assert flags[i] == 0, i
        for sd in (0, 1):
            want = b.dump(sd)
            np.testing.assert_array_equal(dump[i, sd, :len(want)], want, err_msg=f"book {i} side {sd}")
            assert (dump[i, sd, len(want):] == -1).all()


@pytest.mark.parametrize("res", [{"registers": 1}, {"registers": 0}])
def test_episode_from_snapshot_matches_oracle(res):
    n_books, cap, per_step, window_s = 6, 100, 100, 1
    w = W.uniform(n_books, 4000, cap=cap, tag=12)
    start_s = 34201
    ctx = lob.Context(w.caps, l2_levels=LEVELS, trade_log_records=w.caps + 2 * np.diff(w.offs))
    ctx.set_plan(**res)
    wins, steps, firsts = [], [], []
    for i in range(n_books):
        m = w.msgs[w.offs[i]:w.offs[i + 1]]
        win, st, first = lob.windows(m, start_s, window_s, per_step, 16, 1)
        wins.append(win[0])
        steps.append(int(st[0]))
        firsts.append(int(first[0]))
    # replay every book's stream up to its window start, then snapshot
    pre = np.concatenate([w.msgs[w.offs[i]:w.offs[i] + firsts[i]] for i in range(n_books)])
    pre_offs = np.concatenate([[0], np.cumsum(firsts)]).astype(np.int64)
    ctx.process(to_dev(pre), to_dev(pre_offs))
    snap = ctx.read_l2()
    o_pre = O.run(w.caps, pre, pre_offs, l2_mode=O.L2_FINAL, levels=LEVELS)
    np.testing.assert_array_equal(snap.cpu().numpy(), o_pre["l2"])
    # episode: fresh books from the snapshot, then the window's steps
    ep = lob.Context(w.caps, l2_levels=LEVELS, trade_log_records=w.caps + 2 * 16 * per_step)
    ep.set_plan(**res)
    times = np.tile(np.array([[start_s, 0]], np.int32), (n_books, 1))
    ep.seed_l2(snap, times=to_dev(times), init_tid=0)
    books = [oracle_seeded(cap, o_pre["l2"][i], start_s, 0, 0) for i in range(n_books)]
    d_win = to_dev(np.stack(wins))  # [n][16][per_step][8]
    l2 = torch.zeros((n_books, 2, LEVELS, 2), dtype=torch.int32, device="cuda:0")
    for s in range(max(steps)):
        ep.step(d_win[:, s].contiguous(), l2)
        got = l2.cpu().numpy()
        for i in range(n_books):
            for m in wins[i][s]:
                books[i].process(m)
            np.testing.assert_array_equal(got[i], books[i].l2(LEVELS), err_msg=f"book {i} step {s}")
    dump = ep.read_book(cap).cpu().numpy()
    for i in range(n_books):
        for sd in (0, 1):
            want = books[i].dump(sd)
            np.testing.assert_array_equal(dump[i, sd, :len(want)], want)
    # the window's cancels of pre-window orders found seeded orders by price
    st = ep.read_status()
    assert int(st["n_trades"].sum()) > 0
