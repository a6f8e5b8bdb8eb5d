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
def test_exec_steps_match_oracle(res):
    n_books, cap, Wn, n_steps, F = 24, 100, 100, 16, 64
    w = W.uniform(n_books, Wn * n_steps, cap=cap, tag=13)
    seeds = 2 * (cap // 2)
    msgs = w.msgs.reshape(n_books, seeds + Wn * n_steps, 8)
    ctx = lob.Context(w.caps, l2_levels=10, trade_log_records=np.full(n_books, 2 * (Wn + 4) + 8))
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
