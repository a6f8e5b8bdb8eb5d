"""GPU parity: the HIP path (through the C ABI) against the oracle, bit for bit.

Every record is int32, so every comparison is exact: trades per book in order,
final books (canonical priority-ordered dumps), L2 snapshots and counters.
"""
import itertools

import numpy as np
import pytest
import torch

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():  # pragma: no cover - collected on CPU hosts too
    pytest.skip("no GPU", allow_module_level=True)

from golden_cases import all_cases  # noqa: E402
from gpu_helpers import COUNTERS, assert_same, new_context, run_gpu, run_oracle, to_dev  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2308_13289_amd import lob  # noqa: E402
from paper_2308_13289_amd import workload as W  # noqa: E402
from test_oracle_bruteforce import alphabet, to_msgs  # noqa: E402

# The persistent work-queue kernel (device-side longest-first queue built with a
# library radix sort, waves popping books with an atomic counter) faulted the GPU
# on its first run and no defect in this project's code was found by reading it;
# it was withdrawn and ragged batches use lob_process_ragged instead.  Its cases
# stay here, skipped.
WITHDRAWN = pytest.mark.skip(reason="persistent work-queue kernel withdrawn: its first GPU run "
                                    "faulted and the cause was not found")


def test_selftest_primitives():
    out = lob.selftest().cpu().numpy()
    lanes = np.arange(64)
    np.testing.assert_array_equal(out[:64], np.cumsum(lanes % 7 + 1))
    np.testing.assert_array_equal(out[64:128], np.cumsum(lanes % 3 == 0))
    np.testing.assert_array_equal(out[128:192], lanes)
    x = 3 * lanes + 1
    np.testing.assert_array_equal(out[192:256], np.concatenate([[-5], x[:-1]]))
    np.testing.assert_array_equal(out[256:320], np.concatenate([x[1:], [-7]]))
    np.testing.assert_array_equal(out[320:384], x[(lanes + 5) % 64])
    np.testing.assert_array_equal(out[384:448], np.concatenate([[0], x[:-1]]))
    np.testing.assert_array_equal(out[448:512], np.concatenate([x[1:], [0]]))
    np.testing.assert_array_equal(out[512:576], np.where(lanes == 17, -9, x))


RESIDENCY = {"regs": {"registers": 1}, "lds": {"registers": 0}, "unsorted": {"layout": 1},
             "tail": {"registers": 1}, "tail_shallow": {"registers": 1, "tail_shallow": 1}}


@pytest.mark.parametrize("res", ["regs", "lds", "unsorted", "tail", "tail_shallow"])
def test_golden_cases_on_gpu(res):
    """The hand-worked cases; "tail" adds a book of capacity 300 to the call, which
    puts the register kernel in its TAIL form for every book ("tail_shallow": the
    TAIL form's code for drained books)."""
    cases = all_cases()
    tail = res.startswith("tail")
    caps = np.array([c.cap for c in cases] + ([300] if tail else []), np.int32)
    msgs = np.concatenate([c.msgs for c in cases])
    offs = np.concatenate([[0], np.cumsum([len(c.msgs) for c in cases])] +
                          ([[len(msgs)]] if tail else [])).astype(np.int64)
    g = run_gpu(caps, msgs, offs, levels=3, l2_mode=lob.L2_FINAL, plan=RESIDENCY[res])
    for i, c in enumerate(cases):
        tr = g["trades"][g["trade_offs"][i]:g["trade_offs"][i + 1]]
        np.testing.assert_array_equal(tr, c.trades[:, 1:].astype(np.int32), err_msg=c.name)
        d = g["dumps"][i]
        np.testing.assert_array_equal(d[0][:len(c.ask)], c.ask, err_msg=c.name)
        np.testing.assert_array_equal(d[1][:len(c.bid)], c.bid, err_msg=c.name)
        assert (d[0][len(c.ask):] == -1).all() and (d[1][len(c.bid):] == -1).all(), c.name
        if c.l2ask is not None:
            np.testing.assert_array_equal(g["l2"][i][0], c.l2ask, err_msg=c.name)
        if c.l2bid is not None:
            np.testing.assert_array_equal(g["l2"][i][1], c.l2bid, err_msg=c.name)
        for k, v in c.stats.items():
            assert g["status"][k][i] == v, (c.name, k)


@pytest.mark.parametrize("res", ["regs", "lds"])
@pytest.mark.parametrize("cap", [1, 2])
def test_bruteforce_sequences_on_gpu(cap, res):
    streams = [to_msgs(s) for s in itertools.product(alphabet(), repeat=3)]
    msgs = np.array([m for s in streams for m in s], np.int32)
    offs = np.concatenate([[0], np.cumsum([len(s) for s in streams])]).astype(np.int64)
    caps = np.full(len(streams), cap, np.int32)
    g = run_gpu(caps, msgs, offs, levels=2, l2_mode=lob.L2_PER_MESSAGE, plan=RESIDENCY[res])
    o = run_oracle(caps, msgs, offs, levels=2, l2_mode=O.L2_PER_MESSAGE)
    assert_same(g, o, f"brute force cap {cap}")


@pytest.mark.parametrize("res", ["regs", "lds"])
def test_c0_full_parity_per_message_l2(res):
    """64 books x (100 seeds + 1000 messages), capacity 100, L2 after every message."""
    w = W.c0()
    g = run_gpu(w.caps, w.msgs, w.offs, l2_mode=lob.L2_PER_MESSAGE, plan=RESIDENCY[res])
    o = run_oracle(w.caps, w.msgs, w.offs, l2_mode=O.L2_PER_MESSAGE)
    assert_same(g, o, "c0")
    assert o["stats"]["n_trades"].sum() > 30000


@pytest.mark.parametrize("plan", [
    {"books_per_block": 1},
    {"books_per_block": 8},
    pytest.param({"persistent": 1}, marks=WITHDRAWN),
    {"lds_slots": 64},                      # books past 64 orders spill to HBM
    pytest.param({"lds_slots": 64, "persistent": 1}, marks=WITHDRAWN),
    {"registers": 0, "books_per_block": 8},
    {"registers": 0, "lds_slots": 64},
], ids=["bpb1", "bpb8", "persistent", "spill64", "spill64_persistent", "lds_bpb8", "lds_spill64"])
def test_plans_agree_c0(plan):
    w = W.c0()
    g = run_gpu(w.caps, w.msgs, w.offs, l2_mode=lob.L2_FINAL, plan=plan)
    o = run_oracle(w.caps, w.msgs, w.offs, l2_mode=O.L2_FINAL)
    assert_same(g, o, str(plan))


@pytest.mark.parametrize("plan", [
    {},
    {"lds_slots": 128},
    pytest.param({"persistent": 1}, marks=WITHDRAWN),
    pytest.param({"persistent": 1, "lds_slots": 128, "split_buckets": 1, "lds_slots_big": 1000},
                 marks=WITHDRAWN),
    pytest.param({"persistent": 1, "lds_slots": 128, "split_buckets": 1, "lds_slots_big": 256},
                 marks=WITHDRAWN),
    {"registers": 0},
    {"registers": 0, "lds_slots": 128},
    {"lds_slots": 200},
    {"layout": 1, "books_per_block": 2},
    {"tail_shallow": 1},
], ids=["default", "spill128", "persistent", "split", "split_spill", "lds", "lds_spill128", "regs_tail200",
        "unsorted", "tail_shallow"])
def test_ragged_mixed_capacities(plan):
    """Capacities {50,100,500,1000} and uneven stream lengths in one call."""
    w = W.ragged(n_books=96, max_flow=4000)
    g = run_gpu(w.caps, w.msgs, w.offs, l2_mode=lob.L2_FINAL, plan=plan)
    o = run_oracle(w.caps, w.msgs, w.offs, l2_mode=O.L2_FINAL)
    assert_same(g, o, f"ragged {plan}")


@pytest.mark.parametrize("plan", [
    {},
    {"ragged_order": 0},
    {"ragged_split": 100, "lds_slots_big": 1000},
    {"ragged_split": 128, "lds_slots_big": 256, "books_per_block": 8, "books_per_block_big": 2},
    {"ragged_split": 64, "lds_slots_big": 64, "lds_slots": 64},
    {"ragged_split": 100, "lds_slots_big": 1000, "tail_shallow": 1},
], ids=["lpt_one_launch", "listed_order", "split_lds", "split_spill", "split_small_windows", "split_tail_shallow"])
def test_process_ragged(plan):
    """lob_process_ragged: longest stream first, capacity buckets on two streams."""
    w = W.ragged(n_books=96, max_flow=4000)
    g = run_gpu(w.caps, w.msgs, w.offs, l2_mode=lob.L2_FINAL, plan=plan, ragged=True)
    o = run_oracle(w.caps, w.msgs, w.offs, l2_mode=O.L2_FINAL)
    assert_same(g, o, f"process_ragged {plan}")


def test_process_ragged_ids_and_per_message_l2():
    """Listed ids in a scrambled order, per-message L2, repeated and bad ids rejected."""
    w = W.ragged(n_books=40, max_flow=1500)
    ctx = new_context(w.caps, 10, np.diff(w.offs), plan={"ragged_split": 100, "lds_slots_big": 512})
    perm = np.random.default_rng(3).permutation(w.n_books).astype(np.int32)
    sel = np.concatenate([np.arange(w.offs[i], w.offs[i + 1]) for i in perm])
    soffs = np.concatenate([[0], np.cumsum(np.diff(w.offs)[perm])]).astype(np.int64)
    l2 = torch.zeros((len(sel), 2, 10, 2), dtype=torch.int32, device="cuda:0")
    ctx.process_ragged(to_dev(w.msgs[sel]), soffs, book_ids_host=perm, l2_mode=lob.L2_PER_MESSAGE,
                       l2_out=l2)
    o = run_oracle(w.caps[perm], w.msgs[sel], soffs, l2_mode=O.L2_PER_MESSAGE)
    np.testing.assert_array_equal(l2.cpu().numpy(), o["l2"])
    bad = perm.copy()
    bad[1] = bad[0]
    with pytest.raises(lob.LobError):
        ctx.process_ragged(to_dev(w.msgs[sel]), soffs, book_ids_host=bad)
    bad[1] = w.n_books
    with pytest.raises(lob.LobError):
        ctx.process_ragged(to_dev(w.msgs[sel]), soffs, book_ids_host=bad)


def test_small_capacity_rejects_and_deep_books():
    """Capacity 8 (sides fill up and reject) and capacity 300 with a one-sided flow
    that keeps > 64 orders resting (multi-chunk shifts, scans and L2)."""
    a = W.uniform(16, 3000, cap=8, tag=90)
    g = run_gpu(a.caps, a.msgs, a.offs, l2_mode=lob.L2_PER_MESSAGE)
    o = run_oracle(a.caps, a.msgs, a.offs, l2_mode=O.L2_PER_MESSAGE)
    assert_same(g, o, "cap 8")
    assert o["stats"]["rejected_qty"].sum() > 0
    rng = np.random.default_rng(7)
    streams = []
    for b in range(16):
        S = 1 if b % 2 == 0 else -1  # the deep side: bids for even books, asks for odd
        ms, t = [], 0
        for k in range(260):  # resting orders at many prices, some repeated
            ms.append([1, S, int(rng.integers(900, 1000)), int(rng.integers(1, 50)), k + 1, 3, 34200, t])
            t += 1
        for k in range(40):  # cancels of live and dead ids (some deep in the side)
            ms.append([2, S, 0, int(rng.integers(1, 30)), int(rng.integers(1, 260)), 3, 34200, t])
            t += 1
        for k in range(6):  # sweeps of many orders, remainders rest on the other side
            ms.append([1, -S, int(rng.integers(900, 1000)), int(rng.integers(50, 3000)), 1000 + k, 4, 34200, t])
            t += 1
        for k in range(30):  # more orders on both sides, then a cancel of a deep one
            ms.append([1, S, int(rng.integers(850, 950)), int(rng.integers(1, 50)), 3000 + k, 3, 34200, t])
            t += 1
        ms.append([3, S, 0, 100, 3005, 3, 34200, t])
        ms.append([4, -S, 0, 5000, 2000, 4, 34200, t + 1])
        streams.append(ms)
    msgs = np.array([m for s in streams for m in s], np.int32)
    offs = np.concatenate([[0], np.cumsum([len(s) for s in streams])]).astype(np.int64)
    caps = np.full(16, 300, np.int32)
    for plan in ({}, {"lds_slots": 64}, {"lds_slots": 200}, {"registers": 0}, {"registers": 0, "lds_slots": 64},
                 {"layout": 1}):
        g = run_gpu(caps, msgs, offs, l2_mode=lob.L2_PER_MESSAGE, plan=plan)
        o = run_oracle(caps, msgs, offs, l2_mode=O.L2_PER_MESSAGE)
        assert_same(g, o, f"deep books {plan}")


def deep_streams(caps, seed):
    """Per book of capacity C: C + 40 resting orders on one side (the last ones
    rejected once it is full), cancels and deletes of live, dead and rejected ids,
    orders at both ends of the side, sweeps and market orders from the other side
    that take up to a tenth of it each (across the register / tail boundary), then
    mixed flow on both sides."""
    rng = np.random.default_rng(seed)
    streams = []
    for b, C in enumerate(caps):
        S = 1 if b % 2 == 0 else -1
        ms, t, oid = [], 0, 0

        def add(T, side, P, Q, o, tid=3):
            nonlocal t
            ms.append([T, side, P, Q, o, tid, 34200 + t // 1000, t % 1000])
            t += 1

        n1 = C + 40
        for _ in range(n1):
            oid += 1
            add(1, S, int(rng.integers(900, 1000)), int(rng.integers(1, 50)), oid)
        for _ in range(min(200, 2 * C + 4)):
            if rng.random() < 0.8:
                add(2, S, 0, int(rng.integers(1, 60)), int(rng.integers(1, n1 + 1)))
            else:
                add(3, S, 0, 100, int(rng.integers(1, n1 + 1)))
        worst, best = (850, 1005) if S == 1 else (1050, 895)
        for k in range(30):
            oid += 1
            add(1, S, worst if k % 2 == 0 else best, int(rng.integers(1, 50)), oid)
        for _ in range(10):
            oid += 1
            add(1, -S, int(rng.integers(900, 1000)), int(rng.integers(C // 2 + 1, 2 * C + 2)), oid, tid=4)
        for _ in range(3):
            oid += 1
            add(4, -S, 0, int(rng.integers(C // 2 + 1, C + 2)), oid, tid=4)
        for _ in range(200):
            r = rng.random()
            if r < 0.6:
                oid += 1
                add(1, int(rng.choice([-1, 1])), int(rng.integers(940, 960)), int(rng.integers(1, 80)), oid)
            else:
                add(2, int(rng.choice([-1, 1])), 0, int(rng.integers(1, 80)), int(rng.integers(1, oid + 1)))
        streams.append(ms)
    msgs = np.array([m for s in streams for m in s], np.int32)
    offs = np.concatenate([[0], np.cumsum([len(s) for s in streams])]).astype(np.int64)
    return np.asarray(caps, np.int32), msgs, offs


@pytest.mark.parametrize("group,plan", [
    ("small", {}),
    ("small", {"registers": 0}),
    ("small", {"layout": 1}),
    ("large", {}),
    ("large", {"registers": 0}),
    ("large", {"registers": 0, "lds_slots": 64}),
    ("large", {"registers": 0, "lds_slots": 1024}),
], ids=["small-regs", "small-lds", "small-unsorted", "large-regs-tail", "large-lds-spill256", "large-lds-spill64",
        "large-lds-spill1024"])
def test_extreme_capacities(group, plan):
    """The smallest capacities, the edges of the register form (64, 128) and of the
    register + tail form (129, 130), and the largest capacity the library accepts,
    with sides filled to capacity and past it; per-message L2."""
    caps = [1, 2, 3, 63, 64, 65, 127, 128] if group == "small" else [129, 130, 1000, 4095, lob.MAX_CAPACITY]
    caps, msgs, offs = deep_streams(caps, seed=11 if group == "small" else 12)
    g = run_gpu(caps, msgs, offs, l2_mode=lob.L2_PER_MESSAGE, plan=plan)
    o = run_oracle(caps, msgs, offs, l2_mode=O.L2_PER_MESSAGE)
    assert_same(g, o, f"{group} {plan}")
    assert (o["stats"]["rejected_qty"] > 0).all() and (o["stats"]["cancel_miss"] > 0).all()


@pytest.mark.parametrize("shallow", [0, 1])
def test_extreme_capacities_ragged(shallow):
    """Both groups in one lob_process_ragged call, split into a register bucket and
    a register + tail bucket (either code of the TAIL form)."""
    caps, msgs, offs = deep_streams([1, 2, 64, 128, 129, 1000, lob.MAX_CAPACITY], seed=13)
    g = run_gpu(caps, msgs, offs, l2_mode=lob.L2_FINAL, plan={"ragged_split": 128, "tail_shallow": shallow},
                ragged=True)
    o = run_oracle(caps, msgs, offs, l2_mode=O.L2_FINAL)
    assert_same(g, o, "extreme ragged")


def test_plans_at_the_largest_capacity():
    """The default plan of a context holding a book of the largest capacity is one
    that lob_set_plan accepts back; the paper-layout form, which keeps a whole book
    in LDS, is refused for such a context instead of being run."""
    ctx = new_context([100, lob.MAX_CAPACITY], 10, [10, 10])
    before = ctx.get_plan().as_dict()
    assert ctx.set_plan().as_dict() == before
    with pytest.raises(lob.LobError):
        ctx.set_plan(layout=1)
    assert ctx.get_plan().as_dict() == before


def test_split_calls_equal_one_call():
    """Book state stays on the device between calls: three calls = one call."""
    w = W.uniform(48, 1500, tag=93)
    g = run_gpu(w.caps, w.msgs, w.offs, l2_mode=lob.L2_PER_MESSAGE, calls=3)
    o = run_oracle(w.caps, w.msgs, w.offs, l2_mode=O.L2_PER_MESSAGE)
    assert_same(g, o, "3 calls")


@pytest.mark.parametrize("cap", [100, 300])
def test_residency_switch_between_calls(cap):
    """Consecutive calls on one context alternate the register kernel (which writes
    each book to its second buffer), the LDS kernel and the unsorted layout (which
    work in place), with a book read in between: the result equals one oracle run."""
    w = W.uniform(24, 1800, cap=cap, tag=95)
    lens = np.diff(w.offs)
    ctx = new_context(w.caps, 10, lens)
    plans = [RESIDENCY["regs"], RESIDENCY["lds"], RESIDENCY["regs"], RESIDENCY["unsorted"], RESIDENCY["regs"],
             RESIDENCY["regs"]]
    calls = len(plans)
    l2 = torch.zeros((w.n_books, 2, 10, 2), dtype=torch.int32, device="cuda:0")
    for c, plan in enumerate(plans):
        ctx.set_plan(**plan)
        lo = w.offs[:-1] + (lens * c) // calls
        hi = w.offs[:-1] + (lens * (c + 1)) // calls
        idx = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)])
        sub_offs = np.concatenate([[0], np.cumsum(hi - lo)]).astype(np.int64)
        ctx.process(to_dev(w.msgs[idx]), to_dev(sub_offs), l2_mode=lob.L2_FINAL, l2_out=l2)
        if c == 2:
            part = O.run(w.caps, w.msgs[np.concatenate([np.arange(a, b) for a, b in zip(w.offs[:-1], hi)])],
                         np.concatenate([[0], np.cumsum(hi - w.offs[:-1])]).astype(np.int64), dumps=True,
                         dump_cap=cap)
            np.testing.assert_array_equal(ctx.read_book(cap).cpu().numpy(), part["dumps"], err_msg="after 3 calls")
    torch.cuda.synchronize()
    o = run_oracle(w.caps, w.msgs, w.offs, l2_mode=O.L2_FINAL)
    st = ctx.read_status()
    total = int(st["log_records"].sum())
    rec, _, toffs = ctx.read_trades(max(total, 1))
    np.testing.assert_array_equal(toffs.cpu().numpy(), o["trade_offs"])
    np.testing.assert_array_equal(rec[:total].cpu().numpy(), o["trades"][:, :6])
    np.testing.assert_array_equal(ctx.read_book(cap).cpu().numpy(), o["dumps"])
    np.testing.assert_array_equal(l2.cpu().numpy(), o["l2"])
    for k in COUNTERS:
        np.testing.assert_array_equal(st[k], o["stats"][k], err_msg=k)


def test_checkpoint_resume():
    """read_book after half of the stream, write_book into a fresh context, finish
    there: the rest of the trades and the final books match the oracle."""
    w = W.uniform(32, 2000, tag=94)
    lens = np.diff(w.offs)
    half = w.offs[:-1] + lens // 2
    first = np.concatenate([np.arange(a, b) for a, b in zip(w.offs[:-1], half)])
    second = np.concatenate([np.arange(a, b) for a, b in zip(half, w.offs[1:])])
    offs1 = np.concatenate([[0], np.cumsum(half - w.offs[:-1])]).astype(np.int64)
    offs2 = np.concatenate([[0], np.cumsum(w.offs[1:] - half)]).astype(np.int64)
    ctx1 = new_context(w.caps, 10, lens)
    ctx1.process(to_dev(w.msgs[first]), to_dev(offs1))
    dump = ctx1.read_book(100)
    ctx2 = new_context(w.caps, 10, lens)
    ctx2.write_book(dump)
    g = run_gpu(w.caps, w.msgs[second], offs2, l2_mode=lob.L2_FINAL, ctx=ctx2)
    o = run_oracle(w.caps, w.msgs, w.offs, l2_mode=O.L2_FINAL)
    np.testing.assert_array_equal(g["dumps"], o["dumps"])
    np.testing.assert_array_equal(g["l2"], o["l2"])
    ofull = O.run(w.caps, w.msgs, w.offs)
    # trades of the second half: the oracle's trades minus those of the first half
    o1 = O.run(w.caps, w.msgs[first], offs1)
    for i in range(w.n_books):
        want = ofull["trades"][ofull["trade_offs"][i] + o1["trade_counts"][i]:ofull["trade_offs"][i + 1], :6]
        got = g["trades"][g["trade_offs"][i]:g["trade_offs"][i + 1]]
        np.testing.assert_array_equal(got, want)
    assert (g["status"]["flags"] & lob.BOOK_BAD_LOAD == 0).all()


def test_read_trades_drains_only_what_fits():
    w = W.uniform(8, 300, tag=95)
    ctx = new_context(w.caps, 10, np.diff(w.offs))
    ctx.process(to_dev(w.msgs), to_dev(w.offs))
    o = O.run(w.caps, w.msgs, w.offs)
    counts = o["trade_counts"]
    k = 3
    room = int(counts[:k].sum()) + 1  # the first 3 books fit, the 4th does not
    rec, cnt, offs = ctx.read_trades(room)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(cnt.cpu().numpy(), counts)
    assert int(offs[-1]) == counts.sum()
    np.testing.assert_array_equal(rec[:int(counts[:k].sum())].cpu().numpy(),
                                  o["trades"][:o["trade_offs"][k], :6])
    st = ctx.read_status()
    assert (st["log_records"][:k] == 0).all()
    np.testing.assert_array_equal(st["log_records"][k:], counts[k:])
    rec2, cnt2, offs2 = ctx.read_trades(int(counts.sum()))
    torch.cuda.synchronize()
    c2 = cnt2.cpu().numpy()
    assert (c2[:k] == 0).all()
    np.testing.assert_array_equal(rec2[:int(c2.sum())].cpu().numpy(), o["trades"][o["trade_offs"][k]:, :6])


def test_trade_log_full_is_flagged():
    w = W.uniform(4, 2000, tag=96)
    ctx = new_context(w.caps, 10, log_room=np.full(4, 50, np.int64))
    ctx.process(to_dev(w.msgs), to_dev(w.offs))
    st = ctx.read_status()
    o = O.run(w.caps, w.msgs, w.offs)
    assert (st["flags"] & lob.BOOK_TRADE_FULL).all()
    np.testing.assert_array_equal(st["log_records"], np.full(4, 50))
    np.testing.assert_array_equal(st["n_trades"], o["trade_counts"])
    rec, _, _ = ctx.read_trades(200)
    torch.cuda.synchronize()
    want = np.concatenate([o["trades"][o["trade_offs"][i]:o["trade_offs"][i] + 50, :6] for i in range(4)])
    np.testing.assert_array_equal(rec[:200].cpu().numpy(), want)


def test_edge_inputs():
    # zero books, books with no messages, padding only, decreasing time
    ctx = new_context([4, 4, 4], 3, log_room=[16, 16, 16])
    ctx.process(to_dev(np.zeros((0, 8), np.int32)), to_dev(np.zeros(1, np.int64)))
    msgs = np.array([[0] * 8, [0, 1, 5, 5, 1, 1, 1, 1],
                     [1, 1, 100, 5, 1, 0, 10, 5], [1, 1, 101, 5, 2, 0, 10, 4]], np.int32)
    offs = np.array([0, 0, 2, 4], np.int64)
    ctx.process(to_dev(msgs), to_dev(offs))
    st = ctx.read_status()
    assert list(st["n_msgs"]) == [0, 2, 2]
    assert st["flags"][2] & lob.BOOK_TIME_ORDER and not st["flags"][1]
    np.testing.assert_array_equal(st["n_bid"], [0, 0, 2])
    with pytest.raises(lob.LobError):
        ctx.process(to_dev(msgs), to_dev(np.array([0, 1, 2, 3, 4], np.int64)))  # 4 books > 3


def test_reset_and_book_ids_subset():
    w = W.uniform(16, 800, tag=97)
    ctx = new_context(w.caps, 10, np.diff(w.offs) * 2)
    ids = np.arange(1, 16, 2, dtype=np.int32)
    sel = np.concatenate([np.arange(w.offs[i], w.offs[i + 1]) for i in ids])
    soffs = np.concatenate([[0], np.cumsum(np.diff(w.offs)[ids])]).astype(np.int64)
    ctx.process(to_dev(w.msgs[sel]), to_dev(soffs), book_ids=to_dev(ids))
    st = ctx.read_status()
    assert (st["n_msgs"][ids] > 0).all() and (st["n_msgs"][ids - 1] == 0).all()
    ctx.reset()
    st = ctx.read_status()
    assert (st["n_msgs"] == 0).all() and (st["n_bid"] == 0).all() and (st["log_records"] == 0).all()
    g = run_gpu(w.caps, w.msgs, w.offs, l2_mode=lob.L2_FINAL, ctx=ctx)
    o = run_oracle(w.caps, w.msgs, w.offs, l2_mode=O.L2_FINAL)
    assert_same(g, o, "after reset")


@WITHDRAWN
def test_deterministic_repeat():
    w = W.ragged(n_books=64, max_flow=3000)
    a = run_gpu(w.caps, w.msgs, w.offs, l2_mode=lob.L2_FINAL, plan={"persistent": 1})
    b = run_gpu(w.caps, w.msgs, w.offs, l2_mode=lob.L2_FINAL, plan={"persistent": 1})
    for k in ("trades", "trade_offs", "dumps", "l2"):
        np.testing.assert_array_equal(a[k], b[k])


def test_deterministic_repeat_ragged():
    w = W.ragged(n_books=64, max_flow=3000)
    plan = {"ragged_split": 100, "lds_slots_big": 256}
    a = run_gpu(w.caps, w.msgs, w.offs, l2_mode=lob.L2_FINAL, plan=plan, ragged=True)
    b = run_gpu(w.caps, w.msgs, w.offs, l2_mode=lob.L2_FINAL, plan=plan, ragged=True)
    for k in ("trades", "trade_offs", "dumps", "l2"):
        np.testing.assert_array_equal(a[k], b[k])


def test_autotune_ragged_keeps_results_exact():
    """The autotuner only changes speed: after it installs its plan, a ragged run is
    still bit-exact, and the tuned books start from empty."""
    w = W.ragged(n_books=64, max_flow=3000)
    ctx = new_context(w.caps, 10, np.diff(w.offs))
    plan, ms = ctx.autotune_ragged(to_dev(w.msgs), w.offs, max_trials=10)
    assert ms > 0 and plan["books_per_block"] >= 1
    st = ctx.read_status()
    assert (st["n_msgs"] == 0).all() and (st["log_records"] == 0).all()
    g = run_gpu(w.caps, w.msgs, w.offs, l2_mode=lob.L2_FINAL, ctx=ctx, ragged=True)
    o = run_oracle(w.caps, w.msgs, w.offs, l2_mode=O.L2_FINAL)
    assert_same(g, o, f"after autotune {plan}")
    # a listed id out of range is refused before anything runs; the plan stays
    before = ctx.get_plan().as_dict()
    with pytest.raises(lob.LobError) as e:
        ctx.autotune_ragged(to_dev(w.msgs), w.offs[:3], book_ids_host=np.array([0, 64], np.int32), max_trials=2)
    assert e.value.status == lob.EINVAL and ctx.get_plan().as_dict() == before


@pytest.mark.parametrize("res", ["regs", "lds", "unsorted"])
def test_plan_max_capacity_bounds_the_launch(res):
    """Plan max_capacity sizes lob_process_messages launches for the listed books:
    books within the bound give the oracle's results; a listed book above it is
    left untouched and flagged LOB_BOOK_BAD_LOAD."""
    w = W.ragged(n_books=24, max_flow=1500)
    caps = w.caps.copy()
    lens = np.diff(w.offs)
    bound = 100
    small = np.nonzero(caps <= bound)[0].astype(np.int32)
    big = np.nonzero(caps > bound)[0].astype(np.int32)
    assert len(small) and len(big)
    ctx = new_context(caps, 10, lens, plan=dict(RESIDENCY[res], max_capacity=bound))
    listed = np.concatenate([small, big[:1]]).astype(np.int32)
    sel = np.concatenate([np.arange(w.offs[i], w.offs[i + 1]) for i in listed])
    offs = np.concatenate([[0], np.cumsum(lens[listed])]).astype(np.int64)
    l2 = torch.zeros((len(listed), 2, 10, 2), dtype=torch.int32, device="cuda:0")
    ctx.process(to_dev(w.msgs[sel]), to_dev(offs), book_ids=to_dev(listed), l2_mode=lob.L2_FINAL, l2_out=l2)
    st = ctx.read_status()
    assert st["flags"][big[0]] & lob.BOOK_BAD_LOAD
    assert st["n_msgs"][big[0]] == 0 and st["n_ask"][big[0]] == 0 and st["n_bid"][big[0]] == 0
    o = run_oracle(caps[small], w.msgs[np.concatenate([np.arange(w.offs[i], w.offs[i + 1]) for i in small])],
                   np.concatenate([[0], np.cumsum(lens[small])]).astype(np.int64), l2_mode=O.L2_FINAL)
    np.testing.assert_array_equal(l2.cpu().numpy()[:len(small)], o["l2"])
    book = ctx.read_book(int(caps.max()), book_ids=to_dev(small)).cpu().numpy()
    np.testing.assert_array_equal(book[:, :, :o["dumps"].shape[2]], o["dumps"])
    assert (book[:, :, o["dumps"].shape[2]:] == -1).all()
    for k in COUNTERS:
        np.testing.assert_array_equal(st[k][small], o["stats"][k], err_msg=k)
    ctx.close()
