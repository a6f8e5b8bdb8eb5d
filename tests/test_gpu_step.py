"""Environment-step form (lob_step) against the oracle, eager and as a captured
HIP graph.

One step of a book = its 100-message data window, then up to 4 agent orders
(trader id -1), then its L2 snapshot and the step's agent fills (Section 5.1.3:
actions become messages, the data window is fetched, everything is processed).
The oracle sees each book as one stream: initial orders, then window + agent
orders of every step; the snapshot after a step is the per-message L2 row of the
step's last message, and the agent fills are the trades produced by the step's
messages in which either side carries trader id -1.
"""
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

AGENT = -1


def step_case(n_books, n_steps, window=100, cap=100):
    w = W.step_workload(n_books=n_books, n_steps=n_steps, window=window, cap=cap)
    seeds = w.extra["seed_msgs"]
    allm = w.msgs.reshape(n_books, seeds + n_steps * window, 8)
    seed_blk = np.ascontiguousarray(allm[:, :seeds])
    windows = np.ascontiguousarray(allm[:, seeds:].reshape(n_books, n_steps, window, 8))
    actions = w.extra["actions"]
    return w, seed_blk, windows, actions


def oracle_steps(caps, seed_blk, windows, actions, levels=10):
    """Per-step L2 [steps][n][2][L][2], agent fills (list per step per book) from
    the oracle run over each book's concatenated stream."""
    n, steps = windows.shape[0], windows.shape[1]
    streams, ends = [], np.zeros((n, steps), np.int64)
    begs = np.zeros((n, steps), np.int64)
    pos = 0
    for b in range(n):
        parts = [seed_blk[b]]
        pos += len(seed_blk[b])
        for s in range(steps):
            act = actions[b, s][actions[b, s, :, 0] != 0]
            begs[b, s] = pos
            parts += [windows[b, s], act]
            pos += len(windows[b, s]) + len(act)
            ends[b, s] = pos - 1
        streams.append(np.concatenate(parts))
    msgs = np.concatenate(streams)
    offs = np.concatenate([[0], np.cumsum([len(x) for x in streams])]).astype(np.int64)
    r = O.run(caps, msgs, offs, l2_mode=O.L2_PER_MESSAGE, levels=levels)
    l2 = r["l2"][ends.T]  # [steps][n][2][L][2]
    fills = [[None] * n for _ in range(steps)]
    for b in range(n):
        tr = r["trades"][r["trade_offs"][b]:r["trade_offs"][b + 1]]
        tm = r["trade_msg"][r["trade_offs"][b]:r["trade_offs"][b + 1]]
        ag = (tr[:, 6] == AGENT) | (tr[:, 7] == AGENT)
        for s in range(steps):
            sel = ag & (tm >= begs[b, s]) & (tm <= ends[b, s])
            fills[s][b] = tr[sel, :6]
    return l2, fills


class StepRunner:
    def __init__(self, caps, seed_blk, windows, actions, F=64, levels=10):
        self.n, self.steps = windows.shape[0], windows.shape[1]
        self.ctx = lob.Context(caps, l2_levels=levels, trade_log_records=np.asarray(caps, np.int64) * 2)
        self.seed_msgs = to_dev(seed_blk.reshape(-1, 8))
        self.seed_offs = to_dev(np.arange(self.n + 1, dtype=np.int64) * seed_blk.shape[1])
        self.win = [to_dev(windows[:, s]) for s in range(self.steps)]
        self.act = [to_dev(actions[:, s]) for s in range(self.steps)]
        dev = torch.device("cuda:0")
        self.l2 = torch.zeros((self.steps, self.n, 2, levels, 2), dtype=torch.int32, device=dev)
        self.fills = torch.zeros((self.steps, self.n, F, 6), dtype=torch.int32, device=dev)
        self.counts = torch.zeros((self.steps, self.n), dtype=torch.int32, device=dev)

    def seed(self):
        self.ctx.reset()
        self.ctx.process(self.seed_msgs, self.seed_offs)

    def run_steps(self):
        for s in range(self.steps):
            self.ctx.step(self.win[s], self.l2[s], actions=self.act[s], agent_tid=AGENT,
                          fills=self.fills[s], fill_counts=self.counts[s])

    def run_steps_two_chains(self, side):
        """The steps of each half of the books as a chain of launches on its own
        stream (the first half on the current stream, the second on `side`)."""
        cur = torch.cuda.current_stream()
        half = self.n // 2
        ids = [torch.arange(0, half, dtype=torch.int32, device="cuda:0"),
               torch.arange(half, self.n, dtype=torch.int32, device="cuda:0")]
        fork = torch.cuda.Event()
        fork.record(cur)
        side.wait_event(fork)
        for s in range(self.steps):
            for c, (lo, hi, st) in enumerate(((0, half, cur), (half, self.n, side))):
                self.ctx.step(self.win[s][lo:hi], self.l2[s, lo:hi], actions=self.act[s][lo:hi], book_ids=ids[c],
                              agent_tid=AGENT, fills=self.fills[s, lo:hi], fill_counts=self.counts[s, lo:hi],
                              stream=st)
        join = torch.cuda.Event()
        join.record(side)
        cur.wait_event(join)

    def outputs(self):
        torch.cuda.synchronize()
        return self.l2.cpu().numpy().copy(), self.fills.cpu().numpy().copy(), self.counts.cpu().numpy().copy()


def check_against_oracle(l2, fills, counts, ol2, ofills, F):
    np.testing.assert_array_equal(l2, ol2)
    for s in range(len(ofills)):
        for b in range(len(ofills[s])):
            want = ofills[s][b]
            assert counts[s, b] == len(want), (s, b)
            k = min(F, len(want))
            np.testing.assert_array_equal(fills[s, b, :k], want[:k], err_msg=f"step {s} book {b}")


@pytest.mark.parametrize("cap", [100, 300, 1000], ids=["registers", "tail300", "tail1000"])
def test_step_eager_matches_oracle(cap):
    """Capacity 100 runs the register kernel's fills form; 300 and 1000 the form
    with an LDS tail (a book seeded with cap/2 orders per side)."""
    w, seed_blk, windows, actions = step_case(48, 25, cap=cap)
    F = 64
    R = StepRunner(w.caps, seed_blk, windows, actions, F=F)
    R.seed()
    R.run_steps()
    l2, fills, counts = R.outputs()
    ol2, ofills = oracle_steps(w.caps, seed_blk, windows, actions)
    assert sum(len(f) for st in ofills for f in st) > 100  # the agent does trade
    check_against_oracle(l2, fills, counts, ol2, ofills, F)
    st = R.ctx.read_status()
    assert (st["log_records"] == 0).all()  # steps do not log trades


def test_step_fills_overflow_flagged():
    w, seed_blk, windows, actions = step_case(16, 10)
    F = 1
    R = StepRunner(w.caps, seed_blk, windows, actions, F=F)
    R.seed()
    R.run_steps()
    l2, fills, counts = R.outputs()
    ol2, ofills = oracle_steps(w.caps, seed_blk, windows, actions)
    check_against_oracle(l2, fills, counts, ol2, ofills, F)
    st = R.ctx.read_status()
    many = np.array([max(len(ofills[s][b]) for s in range(10)) > 1 for b in range(16)])
    assert many.any()
    np.testing.assert_array_equal((st["flags"] & lob.BOOK_FILLS_FULL) != 0, many)


def test_step_graph_replays_match_eager():
    """Capture all steps in one graph; restore the seeded books eagerly between
    replays; every replay must equal the eager run and the oracle."""
    w, seed_blk, windows, actions = step_case(32, 12)
    F = 64
    R = StepRunner(w.caps, seed_blk, windows, actions, F=F)
    R.seed()
    R.run_steps()
    eager = R.outputs()
    ol2, ofills = oracle_steps(w.caps, seed_blk, windows, actions)
    check_against_oracle(*eager, ol2, ofills, F)
    R.seed()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        R.run_steps()
    for rep in range(3):
        R.seed()                     # eager work between replays
        R.l2.zero_()
        R.fills.zero_()
        R.counts.zero_()
        torch.cuda.synchronize()
        g.replay()
        got = R.outputs()
        for a, b in zip(got, eager):
            np.testing.assert_array_equal(a, b, err_msg=f"replay {rep}")


def test_step_graph_of_two_chains_matches_eager():
    """The graph as the benchmark builds it: the two halves of the books step in two
    chains of launches on two streams.  Every replay (eager work between them)
    equals the eager run of all books together and the oracle."""
    w, seed_blk, windows, actions = step_case(32, 12)
    F = 64
    R = StepRunner(w.caps, seed_blk, windows, actions, F=F)
    R.seed()
    R.run_steps()
    eager = R.outputs()
    ol2, ofills = oracle_steps(w.caps, seed_blk, windows, actions)
    check_against_oracle(*eager, ol2, ofills, F)
    side = torch.cuda.Stream()
    R.seed()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        R.run_steps_two_chains(side)
    for rep in range(3):
        R.seed()
        R.l2.zero_()
        R.fills.zero_()
        R.counts.zero_()
        torch.cuda.synchronize()
        g.replay()
        got = R.outputs()
        for a, b in zip(got, eager):
            np.testing.assert_array_equal(a, b, err_msg=f"replay {rep}")


def test_step_window_padding_and_no_actions():
    """Zero-padded window rows are skipped; steps without actions (A = 0)."""
    w, seed_blk, windows, actions = step_case(8, 6)
    windows = windows.copy()
    windows[:, 3, 50:] = 0                       # a half-padded window
    no_act = np.zeros_like(actions)
    ctx = lob.Context(w.caps, l2_levels=10, trade_log_records=np.asarray(w.caps, np.int64) * 2)
    ctx.process(to_dev(seed_blk.reshape(-1, 8)), to_dev(np.arange(9, dtype=np.int64) * seed_blk.shape[1]))
    l2 = torch.zeros((6, 8, 2, 10, 2), dtype=torch.int32, device="cuda:0")
    for s in range(6):
        ctx.step(to_dev(windows[:, s]), l2[s])
    torch.cuda.synchronize()
    ol2, _ = oracle_steps(w.caps, seed_blk, windows, no_act)
    np.testing.assert_array_equal(l2.cpu().numpy(), ol2)


@pytest.mark.parametrize("cap", [100, 300], ids=["registers", "tail"])
def test_step_sweeps_store_fills_mid_chunk(cap):
    """A data message that trades with 80 standing orders, more than the 64 trade
    records staged at once (every third standing order is the agent's), and agent
    market orders after it: fills are stored from the middle of a chunk as well as
    at its end, in trade order."""
    n, width = 4, 100
    windows = np.zeros((n, 2, width, 8), np.int32)
    actions = np.zeros((n, 2, 4, 8), np.int32)
    for b in range(n):
        side = -1 if b % 2 == 0 else 1  # the resting side: asks for even books
        t, oid = 0, 1
        for s, (rest, sweep) in enumerate([(90, 80 + b), (70, 66)]):
            for k in range(rest):
                price = 1000 + k if side == -1 else 1000 - k
                tid = AGENT if k % 3 == 0 else 7
                windows[b, s, k] = [1, side, price, 1, oid, tid, 34200, t]
                oid, t = oid + 1, t + 1
            windows[b, s, rest] = [4, -side, 0, sweep, oid, 9, 34200, t]  # a data market order
            oid, t = oid + 1, t + 1
            actions[b, s, 0] = [4, -side, 0, 5 + s, oid, AGENT, 34200, t]
            actions[b, s, 1] = [1, side, 1000, 3, oid + 1, AGENT, 34200, t + 1]
            oid, t = oid + 2, t + 2
    seed_blk = np.zeros((n, 1, 8), np.int32)  # one padding message (type 0) per book
    caps = np.full(n, cap, np.int32)
    F = 64
    R = StepRunner(caps, seed_blk, windows, actions, F=F)
    R.seed()
    R.run_steps()
    l2, fills, counts = R.outputs()
    ol2, ofills = oracle_steps(caps, seed_blk, windows, actions)
    assert min(len(ofills[0][b]) for b in range(n)) > 25  # agent fills on both sides of the sweep
    check_against_oracle(l2, fills, counts, ol2, ofills, F)


@pytest.mark.parametrize("cap", [100, 300], ids=["registers", "tail"])
def test_step_times_out_of_order(cap):
    """In half the books some windows carry their time stamps in reverse order, so
    that from then on times go backwards: among equal prices the earlier time still
    wins (Section 4.1).  Capacity 100 runs the register kernel's timed loop; 300
    hands such books to the LDS engine after each step's launch."""
    w, seed_blk, windows, actions = step_case(32, 12, cap=cap)
    windows = windows.copy()
    for b in range(0, 32, 2):
        for s in range(b % 3, 12, 3):
            windows[b, s, :, 6:8] = windows[b, s, ::-1, 6:8]
    F = 64
    R = StepRunner(w.caps, seed_blk, windows, actions, F=F)
    R.seed()
    R.run_steps()
    l2, fills, counts = R.outputs()
    ol2, ofills = oracle_steps(w.caps, seed_blk, windows, actions)
    check_against_oracle(l2, fills, counts, ol2, ofills, F)
    st = R.ctx.read_status()
    flagged = (st["flags"] & lob.BOOK_TIME_ORDER) != 0
    assert flagged[::2].all() and not flagged[1::2].any()
