"""Execution-environment step (lob_exec_step, JAX-LOB Section 5.2) against the
oracle's ExecEnv: per step the observation vector, agent fills and task state
equal exactly; the float64 reward is computed on both sides from the same exact
int64 sums by the same operation sequence without fused operations, so it is
compared for equality too.  Covers buy and sell tasks, empty and full actions,
the forced market order before the episode end, and both kernel residencies."""
import numpy as np
import pytest
import torch

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_helpers import to_dev  # noqa: E402
from oracle import oracle as O  # noqa: E402
from oracle.exec_env import ExecEnv  # noqa: E402
from paper_2308_13289_amd import lob  # noqa: E402
from paper_2308_13289_amd import workload as W  # noqa: E402

AGENT = -1


@pytest.mark.parametrize("res", [{"registers": 1}, {"registers": 0}, {"layout": 1}])
@pytest.mark.parametrize("cap,reverse", [(100, False), (100, True), (300, True)])
def test_exec_steps_match_oracle(res, cap, reverse):
    """reverse: in every other book, every third window carries its time stamps in
    reverse order, so that the book's times go backwards (Section 4.1 time priority):
    capacity 100 runs the register kernel's timed loop, which writes the level-1 rows
    too; capacity 300 hands such books to the LDS engine after the launch."""
    n_books, Wn, n_steps, F = 24, 100, 16, 64
    w = W.uniform(n_books, Wn * n_steps, cap=cap, tag=13)
    seeds = 2 * (cap // 2)
    msgs = w.msgs.reshape(n_books, seeds + Wn * n_steps, 8).copy()
    if reverse:
        for b in range(0, n_books, 2):
            for k in range(b % 3, n_steps, 3):
                blk = msgs[b, seeds + k * Wn:seeds + (k + 1) * Wn]
                blk[:, 6:8] = blk[::-1, 6:8].copy()
    ctx = lob.Context(w.caps, l2_levels=10, trade_log_records=np.full(n_books, 2 * (Wn + 4) + 2 * cap))
    ctx.set_plan(**res)
    ctx.process(to_dev(msgs[:, :seeds].reshape(-1, 8)), to_dev(np.arange(n_books + 1, dtype=np.int64) * seeds))
    rng = np.random.default_rng(3)
    state = np.zeros(n_books, lob.EXEC_STATE_DTYPE)
    envs = []
    start = msgs[:, seeds, 6:8]
    for i in range(n_books):
        b = O.Book(cap)
        for m in msgs[i, :seeds]:
            b.process(m)
        ask, bid = b.dump(0)[0, 0], b.dump(1)[0, 0]
        s = state[i]
        s["task_side"] = 1 if i % 2 else -1
        s["task_qty"] = int(rng.integers(300, 2000))
        s["p_init"] = (int(ask) + int(bid)) // 2
        s["start_s"], s["start_ns"] = int(start[i, 0]), int(start[i, 1])
        s["end_s"] = int(start[i, 0]) + 61  # the forced market order comes about 1 s in
        s["next_oid"] = 1_000_000
        envs.append(ExecEnv(b, s["task_side"], s["task_qty"], s["p_init"], tuple(start[i]), s["end_s"],
                            s["next_oid"], tick=100, passive_ticks=2, agent_tid=AGENT, lam=0.3))
    d_state = torch.from_numpy(state.view(np.uint8)).cuda()
    obs = torch.zeros((n_books, 6 * Wn + 8), dtype=torch.int32, device="cuda:0")
    reward = torch.zeros(n_books, dtype=torch.float64, device="cuda:0")
    fills = torch.zeros((n_books, F, 6), dtype=torch.int32, device="cuda:0")
    counts = torch.zeros(n_books, dtype=torch.int32, device="cuda:0")
    forced = 0
    for k in range(n_steps):
        win = msgs[:, seeds + k * Wn:seeds + (k + 1) * Wn]
        act = rng.integers(-20, 60, (n_books, 4)).astype(np.int32)
        act[k % n_books] = 0
        ctx.exec_step(to_dev(win), to_dev(act), d_state, obs, reward, fills, counts, tick=100, passive_ticks=2,
                      agent_tid=AGENT, lam=0.3)
        g_obs, g_rew = obs.cpu().numpy(), reward.cpu().numpy()
        g_fills, g_counts = fills.cpu().numpy(), counts.cpu().numpy()
        g_state = d_state.cpu().numpy().view(lob.EXEC_STATE_DTYPE)
        for i, env in enumerate(envs):
            was_forced = not env.done and win[i, -1, 6] >= env.end_s - 60
            o_obs, o_rew, o_fills = env.step(win[i], act[i])
            forced += was_forced
            np.testing.assert_array_equal(g_obs[i], o_obs, err_msg=f"obs book {i} step {k}")
            assert g_rew[i] == o_rew, (i, k, g_rew[i], o_rew)
            assert g_counts[i] == len(o_fills), (i, k)
            np.testing.assert_array_equal(g_fills[i, :len(o_fills)], o_fills)
            gs = g_state[i]
            assert (gs["exec_qty"], gs["revenue"], gs["done"], gs["next_oid"], gs["flags"]) == \
                (env.exec_qty, env.revenue, env.done, env.next_oid, 0), (i, k)
    assert forced > 0
    dump = ctx.read_book(cap).cpu().numpy()
    for i, env in enumerate(envs):
        for sd in (0, 1):
            want = env.book.dump(sd)
            np.testing.assert_array_equal(dump[i, sd, :len(want)], want)
    # the steps' trades left the log (keep_trades off)
    assert (ctx.read_status()["log_records"] == 0).all()
    if reverse:
        assert ((ctx.read_status()["flags"] & lob.BOOK_TIME_ORDER) != 0)[::2].all()



@pytest.mark.parametrize("res", [{"registers": 1}, {"registers": 0}, {"layout": 1}])
@pytest.mark.parametrize("F", [8, 2 * 100 + 50 + 4])
def test_exec_step_more_fills_than_buffer(res, F):
    """Step 1 rests an agent order of 1000 at the mid price, inside the spread; step 2's
    50 data market orders of 1 share each all fill against it: 50 agent fills.  With F
    at the bound of lob.h (2 * capacity + W + 4) every result equals the oracle's;
    with F = 8 a task of 5 shares, finished by the first 5 fills, is still exact, and
    a task the first 8 fills leave unfinished is flagged LOB_EXEC_FILLS_MISSING with
    Q_exec and the revenue of those 8 fills."""
    n_books, cap, Wn = 8, 100, 50
    w = W.uniform(n_books, 1, cap=cap, tag=31)
    seeds = 2 * (cap // 2)
    seed_msgs = w.msgs.reshape(n_books, seeds + 1, 8)[:, :seeds]
    ctx = lob.Context(w.caps, l2_levels=10, trade_log_records=np.full(n_books, 2 * (Wn + 4) + 2 * cap))
    ctx.set_plan(**res)
    ctx.process(to_dev(seed_msgs.reshape(-1, 8)), to_dev(np.arange(n_books + 1, dtype=np.int64) * seeds))
    state = np.zeros(n_books, lob.EXEC_STATE_DTYPE)
    envs = []
    win1 = np.zeros((n_books, Wn, 8), np.int32)
    win2 = np.zeros((n_books, Wn, 8), np.int32)
    for i in range(n_books):
        b = O.Book(cap)
        for m in seed_msgs[i]:
            b.process(m)
        ask, bid = b.dump(0)[0, 0], b.dump(1)[0, 0]
        s = state[i]
        side = 1 if i % 2 else -1
        s["task_side"] = side
        s["task_qty"] = 1_000_000_000 if i % 4 < 2 else 5
        s["p_init"] = (int(ask) + int(bid)) // 2
        s["start_s"], s["start_ns"] = 34200, 0
        s["end_s"] = 40000
        s["next_oid"] = 1_000_000
        # step 1: one cancel that finds nothing (it sets the step's time); step 2:
        # market orders of 1 share against the agent's side
        win1[i, 0] = [2, 1, 1, 1, 999_999, 7, 34200, 0]
        for k in range(Wn):
            win2[i, k] = [4, -side, 0, 1, 2000 + k, 7, 34200, 1 + k]
        envs.append(ExecEnv(b, side, s["task_qty"], s["p_init"], (34200, 0), s["end_s"], s["next_oid"], tick=100,
                            passive_ticks=2, agent_tid=AGENT, lam=0.3))
    d_state = torch.from_numpy(state.view(np.uint8)).cuda()
    obs = torch.zeros((n_books, 6 * Wn + 8), dtype=torch.int32, device="cuda:0")
    reward = torch.zeros(n_books, dtype=torch.float64, device="cuda:0")
    fills = torch.zeros((n_books, F, 6), dtype=torch.int32, device="cuda:0")
    counts = torch.zeros(n_books, dtype=torch.int32, device="cuda:0")
    acts = [np.tile(np.array([0, 1000, 0, 0], np.int32), (n_books, 1)), np.zeros((n_books, 4), np.int32)]
    flagged = 0
    for step, (win, act) in enumerate(zip([win1, win2], acts)):
        ctx.exec_step(to_dev(win), to_dev(act), d_state, obs, reward, fills, counts, tick=100, passive_ticks=2,
                      agent_tid=AGENT, lam=0.3)
        g_state = d_state.cpu().numpy().view(lob.EXEC_STATE_DTYPE)
        g_counts, g_fills, g_obs, g_rew = counts.cpu().numpy(), fills.cpu().numpy(), obs.cpu().numpy(), \
            reward.cpu().numpy()
        for i, env in enumerate(envs):
            before = env.exec_qty
            o_obs, o_rew, o_fills = env.step(win[i], act[i])
            assert g_counts[i] == len(o_fills), (step, i)
            assert step == 0 or len(o_fills) == Wn, (i, len(o_fills))
            np.testing.assert_array_equal(g_fills[i, :min(F, len(o_fills))], o_fills[:F])
            np.testing.assert_array_equal(g_obs[i, :-1], o_obs[:-1])  # the last entry is Q_exec
            gs = g_state[i]
            # Q_exec and revenue over the first F fills, capped at the task size
            first, rev = before, 0
            for f in o_fills[:F]:
                take = min(int(f[1]), env.task_qty - first)
                if take > 0:
                    first += take
                    rev += take * int(f[0])
            if len(o_fills) > F and first < env.task_qty:
                flagged += 1
                assert gs["flags"] == lob.EXEC_FILLS_MISSING, (step, i)
                assert (gs["exec_qty"], gs["revenue"]) == (first, rev), (step, i)
            else:
                assert gs["flags"] == 0, (step, i)
                assert (gs["exec_qty"], gs["revenue"], gs["done"]) == (env.exec_qty, env.revenue, env.done), i
                assert g_obs[i, -1] == o_obs[-1] and g_rew[i] == o_rew, (step, i)
    assert flagged == (n_books // 2 if F == 8 else 0)


def deep_level_books(cap, depths, rng):
    """Seeds and flow for books whose best level holds d orders on each side (d up to
    the capacity); one side's orders of 2^29 shares (4 or more sum past INT32_MAX), the
    other's of about a thousand, alternating by book.  The flow cancels best-level
    orders (in part or whole), adds to the best levels, trades against them and rests
    one tick behind them, so depth, sum and price of level 1 change message by message."""
    big = 1 << 29
    pa, pb = 1_000_000, 990_000
    seeds, flows = [], []
    for i, d in enumerate(depths):
        t = [34200, 0]

        def tick():
            t[1] += 1
            return list(t)
        qs = {-1: big, 1: 1000} if i % 2 == 0 else {-1: 1000, 1: big}
        book, oids = [], {-1: [], 1: []}
        for sd, p0, step in ((-1, pa, 100), (1, pb, -100)):
            for k in range(d):
                oid = 10_000 * (2 + sd) + k
                oids[sd].append(oid)
                book.append([1, sd, p0, qs[sd] + (k % 7), oid, 7] + tick())
            for k in range(min(cap - d, 3)):
                book.append([1, sd, p0 + step * (k + 1), qs[sd], 50_000 + 10 * (2 + sd) + k, 7] + tick())
        flow = []
        next_oid = 100_000
        for _ in range(3 * 60):
            sd = int(rng.choice([-1, 1]))
            p0 = pa if sd == -1 else pb
            r = rng.random()
            if r < 0.35:
                oid = int(rng.choice(oids[sd]))
                flow.append([2 if rng.random() < 0.5 else 3, sd, p0, int(rng.choice([100, 1 << 30])), oid, 7] + tick())
            elif r < 0.6:
                flow.append([1, sd, p0, qs[sd], next_oid, 7] + tick())
                oids[sd].append(next_oid)
                next_oid += 1
            elif r < 0.8:
                flow.append([4, -sd, 0, int(0.6 * qs[sd]), next_oid, 7] + tick())
                next_oid += 1
            else:
                flow.append([1, sd, p0 + (100 if sd == -1 else -100), qs[sd], next_oid, 7] + tick())
                next_oid += 1
        seeds.append(np.array(book, np.int32))
        flows.append(np.array(flow, np.int32))
    return seeds, np.stack(flows)


@pytest.mark.parametrize("res", [{"registers": 1}, {"registers": 0}])
@pytest.mark.parametrize("cap", [100, 128, 250])
def test_exec_step_deep_best_level(res, cap):
    """Level-1 rows when the best level holds from 1 order to the whole capacity: a
    level spanning both register chunks and, at capacity 250, the tail; level sums past
    INT32_MAX saturate.  Observation, reward, task state and books equal the oracle's
    after every step (three steps of 60 data messages, no agent orders)."""
    depths = sorted({d for d in (1, 2, 3, 63, 64, 65, 127, 128, 129, 200) if d <= cap} | {cap})
    n_books, Wn, F = len(depths), 60, 16
    rng = np.random.default_rng(cap)
    seeds, flow = deep_level_books(cap, depths, rng)
    ctx = lob.Context(np.full(n_books, cap, np.int32), l2_levels=1,
                      trade_log_records=np.full(n_books, 4 * Wn + 2 * cap + 8))
    ctx.set_plan(**res)
    offs = np.concatenate([[0], np.cumsum([len(s) for s in seeds])]).astype(np.int64)
    ctx.process(to_dev(np.concatenate(seeds)), to_dev(offs))
    state = np.zeros(n_books, lob.EXEC_STATE_DTYPE)
    envs = []
    for i in range(n_books):
        b = O.Book(cap)
        for m in seeds[i]:
            b.process(m)
        s = state[i]
        s["task_side"] = 1 if i % 2 else -1
        s["task_qty"] = 1000
        s["p_init"] = 995_000
        s["start_s"], s["start_ns"] = 34200, 0
        s["end_s"] = 40000
        s["next_oid"] = 1_000_000
        envs.append(ExecEnv(b, s["task_side"], s["task_qty"], s["p_init"], (34200, 0), s["end_s"], s["next_oid"],
                            tick=100, passive_ticks=2, agent_tid=AGENT, lam=0.3))
    d_state = torch.from_numpy(state.view(np.uint8)).cuda()
    obs = torch.zeros((n_books, 6 * Wn + 8), dtype=torch.int32, device="cuda:0")
    reward = torch.zeros(n_books, dtype=torch.float64, device="cuda:0")
    fills = torch.zeros((n_books, F, 6), dtype=torch.int32, device="cuda:0")
    counts = torch.zeros(n_books, dtype=torch.int32, device="cuda:0")
    act = np.zeros((n_books, 4), np.int32)
    saturated = 0
    for k in range(3):
        win = np.ascontiguousarray(flow[:, k * Wn:(k + 1) * Wn])
        ctx.exec_step(to_dev(win), to_dev(act), d_state, obs, reward, fills, counts, tick=100, passive_ticks=2,
                      agent_tid=AGENT, lam=0.3)
        g_obs, g_rew = obs.cpu().numpy(), reward.cpu().numpy()
        g_state = d_state.cpu().numpy().view(lob.EXEC_STATE_DTYPE)
        for i, env in enumerate(envs):
            o_obs, o_rew, _ = env.step(win[i], act[i])
            saturated += int((np.abs(o_obs[5 * Wn:6 * Wn].astype(np.int64)) >= (1 << 31) - (1 << 20)).sum())
            np.testing.assert_array_equal(g_obs[i], o_obs, err_msg=f"obs book {i} (depth {depths[i]}) step {k}")
            assert g_rew[i] == o_rew, (i, k)
            gs = g_state[i]
            assert (gs["exec_qty"], gs["revenue"], gs["done"], gs["flags"]) == \
                (env.exec_qty, env.revenue, env.done, 0), (i, k)
    assert saturated > 0
    dump = ctx.read_book(cap).cpu().numpy()
    for i, env in enumerate(envs):
        for sd in (0, 1):
            want = env.book.dump(sd)
            np.testing.assert_array_equal(dump[i, sd, :len(want)], want, err_msg=f"book {i} side {sd}")
