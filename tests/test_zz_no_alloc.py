"""lob_exec_step_noalloc (its scratch in the library's static array) against
lob_exec_step (its scratch in the context) through the C ABI: two contexts with the
same books take the same steps, one through each entry point, and every output
is compared exactly -- observation, reward, agent fills and their counts, the task
state and the books.  Two calls in a row, the second over fewer books with a
shorter window; capacity 100 (register kernel) and 300 (its TAIL form, whose
per-message rows send books whose times go backwards to the LDS engine)."""
import numpy as np
import pytest
import torch

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_helpers import to_dev  # noqa: E402
from paper_2308_13289_amd import lob  # noqa: E402
from paper_2308_13289_amd import workload as W  # noqa: E402

AGENT = -1


def seeded_pair(n_books, cap, n_flow, tag):
    w = W.uniform(n_books, n_flow, cap=cap, tag=tag)
    seeds = 2 * (cap // 2)
    msgs = w.msgs.reshape(n_books, seeds + n_flow, 8)
    ctxs = []
    for _ in range(2):
        c = lob.Context(w.caps, l2_levels=10, trade_log_records=np.full(n_books, 2 * (n_flow + 4) + cap))
        c.process(to_dev(msgs[:, :seeds].reshape(-1, 8)), to_dev(np.arange(n_books + 1, dtype=np.int64) * seeds))
        ctxs.append(c)
    state = np.zeros(n_books, lob.EXEC_STATE_DTYPE)
    for i in range(n_books):
        s = state[i]
        s["task_side"] = 1 if i % 2 else -1
        s["task_qty"] = 500 + 37 * i
        s["p_init"] = 10_000_000
        s["start_s"], s["start_ns"] = int(msgs[i, seeds, 6]), int(msgs[i, seeds, 7])
        s["end_s"] = int(msgs[i, seeds, 6]) + 3600
        s["next_oid"] = 1_000_000
    return ctxs, msgs[:, seeds:], state


def run(ctx, ids, win, act, state, F, noalloc):
    n, Wn = win.shape[0], win.shape[1]
    dev = torch.device("cuda:0")
    obs = torch.full((n, 6 * Wn + 8), -7, dtype=torch.int32, device=dev)
    reward = torch.full((n,), -7.0, dtype=torch.float64, device=dev)
    fills = torch.full((n, F, 6), -7, dtype=torch.int32, device=dev)
    counts = torch.full((n,), -7, dtype=torch.int32, device=dev)
    ctx.exec_step(to_dev(win), to_dev(act), state, obs, reward, fills, counts, tick=100, passive_ticks=1,
                  agent_tid=AGENT, lam=0.25, book_ids=to_dev(ids), noalloc=noalloc)
    torch.cuda.synchronize()
    return obs.cpu().numpy(), reward.cpu().numpy(), fills.cpu().numpy(), counts.cpu().numpy()


@pytest.mark.parametrize("cap", [100, 300])
def test_noalloc_step_equals_exec_step(cap):
    n_books, F = 40, 32
    (ctx_a, ctx_b), flow, state = seeded_pair(n_books, cap, 150, tag=61)
    st_a = torch.from_numpy(state.view(np.uint8).copy()).cuda()
    st_b = torch.from_numpy(state.view(np.uint8).copy()).cuda()
    rng = np.random.default_rng(9)
    calls = [(np.arange(n_books, dtype=np.int32), flow[:, :100]),
             (np.arange(3, n_books, 2, dtype=np.int32), flow[3::2, 100:150])]
    for ids, win in calls:
        act = rng.integers(-5, 40, (len(ids), 4)).astype(np.int32)
        win = np.ascontiguousarray(win)
        # the state rows of the listed books, in listed order
        sel = torch.from_numpy(ids.astype(np.int64)).cuda()
        rows_a = st_a.view(n_books, 48)[sel].contiguous().view(-1)
        rows_b = st_b.view(n_books, 48)[sel].contiguous().view(-1)
        ra = run(ctx_a, ids, win, act, rows_a, F, noalloc=False)
        rb = run(ctx_b, ids, win, act, rows_b, F, noalloc=True)
        for x, y, name in zip(ra, rb, ["obs", "reward", "fills", "counts"]):
            np.testing.assert_array_equal(x, y, err_msg=name)
        np.testing.assert_array_equal(rows_a.cpu().numpy(), rows_b.cpu().numpy(), err_msg="state")
        assert (ra[3] > 0).any()  # the agent traded
        st_a.view(n_books, 48)[sel] = rows_a.view(len(ids), 48)
        st_b.view(n_books, 48)[sel] = rows_b.view(len(ids), 48)
    np.testing.assert_array_equal(ctx_a.read_book(cap).cpu().numpy(), ctx_b.read_book(cap).cpu().numpy())
    ctx_a.close()
    ctx_b.close()


def test_noalloc_rejects_more_books_than_its_scratch():
    n = lob.NOALLOC_MAX_BOOKS + 1
    ctx = lob.Context(np.ones(n, np.int32), l2_levels=1, trade_log_records=np.full(n, 8))
    dev = torch.device("cuda:0")
    win = torch.zeros((n, 1, 8), dtype=torch.int32, device=dev)
    with pytest.raises(lob.LobError) as e:
        ctx.exec_step(win, torch.zeros((n, 4), dtype=torch.int32, device=dev),
                      torch.zeros(n * 48, dtype=torch.uint8, device=dev),
                      torch.zeros((n, 14), dtype=torch.int32, device=dev),
                      torch.zeros(n, dtype=torch.float64, device=dev),
                      torch.zeros((n, 1, 6), dtype=torch.int32, device=dev),
                      torch.zeros(n, dtype=torch.int32, device=dev), noalloc=True)
    assert e.value.status == lob.ECAP and "LOB_NOALLOC_MAX_BOOKS" in str(e.value)
    ctx.close()
