"""Serving loop (lob_server_*): every request's result equals the oracle's replay
of its book in arrival order, and equals the result of running the same trace
one request at a time (tolerance 0: everything is integer)."""
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
from paper_2308_13289_amd import serve as S  # noqa: E402

LEVELS = 10


def seeded_context(sw, plan=None):
    caps = sw.caps
    room = 2 * caps.astype(np.int64) + 2 * (1000 + 4)
    ctx = lob.Context(caps, l2_levels=LEVELS, trade_log_records=room)
    if plan:
        ctx.set_plan(**plan)
    s0, s1 = sw.seed_offsets
    seeds = np.concatenate([sw.w.msgs[a:b] for a, b in zip(s0, s1)])
    offs = np.concatenate([[0], np.cumsum(s1 - s0)]).astype(np.int64)
    ctx.process(to_dev(seeds), to_dev(offs))
    torch.cuda.synchronize()
    return ctx


def oracle_results(sw, books):
    msgs, offs, spans = sw.oracle_streams(books)
    r = O.run(sw.caps[np.asarray(books)], msgs, offs, l2_mode=O.L2_PER_MESSAGE, levels=LEVELS)
    out = {}
    tm = r["trade_msg"]
    tr = r["trades"]
    for k, first, last in spans:
        sel = (tm >= first) & (tm <= last)
        if sw.kind[k] == S.REPLAY:
            out[k] = ("replay", tr[sel, :6])
        else:
            ag = sel & ((tr[:, 6] == -1) | (tr[:, 7] == -1))
            out[k] = ("step", r["l2"][last], tr[ag, :6])
    return out


def check(sw, comp, want):
    assert len(comp) == sw.n
    assert (comp["status"] == lob.OK).all()
    assert sorted(comp["tag"]) == list(range(sw.n))
    n_out = dict(zip(comp["tag"], comp["n_out"]))
    for k, w in want.items():
        if w[0] == "replay":
            got = sw.trades[sw.trade_offs[k]:sw.trade_offs[k] + n_out[k]]
            np.testing.assert_array_equal(got, w[1], err_msg=f"replay request {k}")
        else:
            np.testing.assert_array_equal(sw.l2[k], w[1], err_msg=f"step request {k} L2")
            assert n_out[k] == len(w[2]), k
            np.testing.assert_array_equal(sw.fills[k][:n_out[k]], w[2], err_msg=f"step request {k} fills")


def test_serving_matches_oracle_in_arrival_order():
    sw = S.ServingWorkload(n_books=300, lam=40_000, duration_s=0.05)
    assert sw.n > 1000 and (sw.kind == S.STEP).any() and (sw.kind == S.REPLAY).any()
    ctx = seeded_context(sw, plan={"lds_slots": 128})
    srv = S.Server(ctx, n_slots=4, hbm_budget=256 << 20, max_batch=512)
    comp = srv.run(sw.requests(), sw.arrival)
    want = oracle_results(sw, list(range(300)))
    check(sw, comp, want)
    lat = comp["complete_ns"] - comp["arrival_ns"]
    assert (lat > 0).all() and (comp["launch_ns"] >= comp["arrival_ns"]).all()
    srv.close()


def test_alone_equals_mixed():
    """The same trace with one request per batch and one slot (each request alone on
    the GPU) gives exactly the results of the mixed, batched run."""
    sw = S.ServingWorkload(n_books=120, lam=30_000, duration_s=0.03)
    ctx = seeded_context(sw)
    comp = S.Server(ctx, n_slots=4, hbm_budget=128 << 20, max_batch=256).run(sw.requests(), sw.arrival)
    mixed = (sw.trades.copy(), sw.l2.copy(), sw.fills.copy(), dict(zip(comp["tag"], comp["n_out"])))
    sw.trades[:] = 0
    sw.l2[:] = 0
    sw.fills[:] = 0
    ctx2 = seeded_context(sw)
    comp2 = S.Server(ctx2, n_slots=1, hbm_budget=64 << 20, max_batch=1).run(sw.requests(),
                                                                              np.zeros(sw.n, np.int64))
    assert dict(zip(comp2["tag"], comp2["n_out"])) == mixed[3]
    np.testing.assert_array_equal(sw.trades, mixed[0])
    np.testing.assert_array_equal(sw.l2, mixed[1])
    np.testing.assert_array_equal(sw.fills, mixed[2])


def test_tight_budget_waits_not_fails():
    """A budget that holds only a few requests per batch: everything still completes,
    in more batches, with the same results."""
    sw = S.ServingWorkload(n_books=60, lam=20_000, duration_s=0.02)
    ctx = seeded_context(sw)
    # room for about one 1000-message request per slot
    srv = S.Server(ctx, n_slots=2, hbm_budget=2 * 400_000, max_batch=64)
    comp = srv.run(sw.requests(), sw.arrival)
    check(sw, comp, oracle_results(sw, list(range(60))))


def test_bad_requests_rejected():
    sw = S.ServingWorkload(n_books=10, lam=10_000, duration_s=0.002)
    ctx = seeded_context(sw)
    srv = S.Server(ctx, n_slots=1, hbm_budget=64 << 20, max_batch=8)
    R = sw.requests()
    R[0].book = 10
    with pytest.raises(lob.LobError):
        srv.run(R, sw.arrival)
    with pytest.raises(lob.LobError):
        S.Server(ctx, n_slots=1, hbm_budget=1000, max_batch=8)
