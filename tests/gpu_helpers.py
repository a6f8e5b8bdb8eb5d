"""Helpers for the GPU parity tests: run a workload through liblob (C ABI) and
through the oracle, and compare."""
import numpy as np
import torch

from oracle import oracle as O
from paper_2308_13289_amd import lob


def dev():
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def new_context(caps, levels=10, msgs_per_book=None, plan=None, log_room=None):
    """Context whose trade logs hold the closed-form bound for the given streams
    (or log_room records per book)."""
    caps = np.asarray(caps, np.int32)
    if log_room is None:
        if msgs_per_book is None:
            log_room = np.full(len(caps), 0, np.int64)
        else:
            log_room = np.asarray(caps, np.int64) + 2 * np.asarray(msgs_per_book, np.int64)
    ctx = lob.Context(caps, l2_levels=levels, trade_log_records=np.asarray(log_room, np.int64))
    if plan:
        ctx.set_plan(**plan)
    return ctx


def run_gpu(caps, msgs, offs, levels=10, l2_mode=lob.L2_NONE, plan=None, ctx=None, calls=1,
            ragged=False):
    """Process every book's stream (optionally split into `calls` consecutive calls)
    and read back trades, L2, final books and counters."""
    caps = np.asarray(caps, np.int32)
    offs = np.asarray(offs, np.int64)
    n = len(caps)
    if ctx is None:
        ctx = new_context(caps, levels, np.diff(offs), plan)
    d_msgs = to_dev(msgs)
    l2 = None
    if l2_mode == lob.L2_PER_MESSAGE:
        l2 = torch.zeros((msgs.shape[0], 2, levels, 2), dtype=torch.int32, device=dev())
    elif l2_mode == lob.L2_FINAL:
        l2 = torch.zeros((n, 2, levels, 2), dtype=torch.int32, device=dev())
    lens = np.diff(offs)
    for c in range(calls):
        lo = offs[:-1] + (lens * c) // calls
        hi = offs[:-1] + (lens * (c + 1)) // calls
        # one call: listed book i reads msgs[lo[i]:hi[i]); offsets must be monotone,
        # so give each call its own gathered message array
        idx = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)]) if n else np.zeros(0, np.int64)
        sub_offs = np.concatenate([[0], np.cumsum(hi - lo)]).astype(np.int64)
        sub = torch.from_numpy(np.ascontiguousarray(msgs[idx] if len(idx) else np.zeros((0, 8), np.int32)))
        d_sub = sub.to(dev()) if calls > 1 else d_msgs
        mode = l2_mode
        out = l2
        if l2_mode == lob.L2_PER_MESSAGE and calls > 1:
            out = torch.zeros((max(len(idx), 1), 2, levels, 2), dtype=torch.int32, device=dev())
        if ragged:
            ctx.process_ragged(d_sub, sub_offs, l2_mode=mode, l2_out=out)
        else:
            ctx.process(d_sub, to_dev(sub_offs), l2_mode=mode, l2_out=out)
        if l2_mode == lob.L2_PER_MESSAGE and calls > 1 and len(idx):
            l2[torch.from_numpy(idx).to(dev())] = out[:len(idx)]
    torch.cuda.synchronize()
    st = ctx.read_status()
    total = int(st["log_records"].sum())
    rec, counts, toffs = ctx.read_trades(max(total, 1))
    torch.cuda.synchronize()
    dumps = ctx.read_book(int(caps.max()))
    res = {
        "trades": rec[:total].cpu().numpy(),
        "trade_offs": toffs.cpu().numpy(),
        "trade_counts": counts.cpu().numpy(),
        "status": st,
        "l2": None if l2 is None else l2.cpu().numpy(),
        "dumps": dumps.cpu().numpy(),
        "ctx": ctx,
    }
    return res


def run_oracle(caps, msgs, offs, levels=10, l2_mode=O.L2_NONE):
    caps = np.asarray(caps, np.int32)
    return O.run(caps, msgs, offs, l2_mode=l2_mode, levels=levels, dumps=True, dump_cap=int(caps.max()))


COUNTERS = ["n_msgs", "n_trades", "limit_qty", "market_qty", "traded_qty", "cancelled_qty",
            "market_discarded", "rejected_qty", "cancel_miss", "flags"]


def assert_same(g, o, what=""):
    """Bit-exact comparison of a GPU run and an oracle run over the same books."""
    np.testing.assert_array_equal(g["trade_offs"], o["trade_offs"], err_msg=f"{what}: trades per book")
    np.testing.assert_array_equal(g["trades"], o["trades"][:, :6], err_msg=f"{what}: trade records")
    np.testing.assert_array_equal(g["dumps"], o["dumps"], err_msg=f"{what}: final books")
    for k in COUNTERS:
        np.testing.assert_array_equal(g["status"][k], o["stats"][k], err_msg=f"{what}: counter {k}")
    if o["l2"] is not None:
        np.testing.assert_array_equal(g["l2"], o["l2"], err_msg=f"{what}: L2")
