"""GPU parity at the edges of the input domain, for every residency form.

* Quantities up to INT32_MAX (Section 4.2 makes Q an int32 field): sweeps whose
  fills add up past INT32_MAX, in one 64-order chunk and across chunks, resting
  quantities far above the aggressor's, and L2 levels whose summed quantity passes
  INT32_MAX (reported capped, as the oracle does).
* Times that repeat and go backwards: among equal prices the earlier (Ts, Tns) has
  priority (Section 4.1), equal times keep arrival order, and the book is flagged.

Residencies: registers (capacity <= 128), registers with an LDS tail (a capacity
of 300 in the same call), the LDS kernel (whole side in LDS, and with slots past 64
spilled to HBM) and the paper's unsorted layout.  Every comparison is bit-exact.
"""
import itertools

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if not gpu_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from gpu_helpers import assert_same, run_gpu, run_oracle  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2308_13289_amd import lob  # noqa: E402
from test_oracle_bruteforce import PREFIX_BIG, alphabet, alphabet_big, to_msgs  # noqa: E402

BIG = 2 ** 31 - 1
PLANS = {"regs": {"registers": 1}, "tail": {"registers": 1}, "tail_shallow": {"registers": 1, "tail_shallow": 1},
         "lds": {"registers": 0},
         "spill": {"registers": 0, "lds_slots": 64}, "unsorted": {"layout": 1}}
# one more book of this capacity in the same call puts the register kernel in its
# TAIL form (and gives the LDS kernels a window past 128)
TAIL_CAP = 300


def with_tail_book(caps, msgs, offs):
    caps = np.concatenate([caps, [TAIL_CAP]]).astype(np.int32)
    offs = np.concatenate([offs, [offs[-1]]]).astype(np.int64)
    return caps, msgs, offs


def compare(caps, msgs, offs, res, levels, l2_mode=lob.L2_PER_MESSAGE, calls=1):
    caps = np.asarray(caps, np.int32)
    offs = np.asarray(offs, np.int64)
    if res.startswith("tail"):
        caps, msgs, offs = with_tail_book(caps, msgs, offs)
    g = run_gpu(caps, msgs, offs, levels=levels, l2_mode=l2_mode, plan=PLANS[res], calls=calls)
    o = run_oracle(caps, msgs, offs, levels=levels, l2_mode=l2_mode)
    assert_same(g, o, res)
    return o


def flow(rng, n_books, n_msgs, cap, big, shuffled_times, mid=10_000_000, tick=100):
    """Synthetic streams: a deep book of resting orders, then limit, market, cancel
    and delete messages.  big: quantities from {1..10, ~2^24, 1e9..INT32_MAX} and, in
    half the books, resting orders of 2e7..4e7 (a market order of INT32_MAX sweeps
    more than 64 of them); shuffled_times: times drawn from a few values, so they
    repeat and go backwards."""
    def qty():
        if not big:
            return int(rng.integers(1, 200))
        k = rng.integers(0, 4)
        if k == 0:
            return int(rng.integers(1, 11))
        if k == 1:
            return int(rng.integers((1 << 24) - 8, (1 << 24) + 8))
        if k == 2:
            return int(rng.integers(1_000_000_000, BIG))
        return BIG

    books = []
    for b in range(n_books):
        msgs, live = [], []
        deep = big and b % 2 == 0
        n_seed = min(cap - 4, 90 if cap <= 128 else cap - 20) // 2 * 2
        oid = 1
        for s in range(n_seed):
            side = 1 if s % 2 else -1
            p = mid - side * tick * (1 + s // 2)
            q = int(rng.integers(20_000_000, 40_000_000)) if deep else qty()
            msgs.append([1, side, p, q, oid, 3, 0, 0])
            live.append((oid, side, p))
            oid += 1
        for _ in range(n_msgs):
            r = rng.random()
            if r < 0.5 or not live:
                side = int(rng.choice([1, -1]))
                p = mid + tick * int(np.round(rng.normal(0, 8)))
                msgs.append([1, side, p, qty(), oid, 4, 0, 0])
                live.append((oid, side, p))
                oid += 1
            elif r < 0.65:
                msgs.append([4, int(rng.choice([1, -1])), 0, qty(), oid, 5, 0, 0])
                oid += 1
            else:
                tid, side, p = live[int(rng.integers(0, len(live)))]
                msgs.append([2 if r < 0.9 else 3, side, p, qty() if r < 0.9 else BIG, tid, 6, 0, 0])
        for k, m in enumerate(msgs):
            if shuffled_times:
                m[6], m[7] = 34200 + int(rng.integers(0, 3)), int(rng.integers(0, 4))
            else:
                m[6], m[7] = 34200 + k // 1000, k % 1000
        books.append(np.array(msgs, np.int32))
    offs = np.concatenate([[0], np.cumsum([len(m) for m in books])]).astype(np.int64)
    return np.full(n_books, cap, np.int32), np.concatenate(books), offs


@pytest.mark.parametrize("res", ["regs", "tail", "tail_shallow", "lds", "unsorted"])
@pytest.mark.parametrize("cap", [2, 3])
def test_bruteforce_large_quantities(cap, res):
    """Every length-3 sequence of the large-quantity alphabet after two initial
    orders of INT32_MAX shares (the oracle's own brute-force pin)."""
    streams = [to_msgs(s, PREFIX_BIG) for s in itertools.product(alphabet_big(), repeat=3)]
    msgs = np.array([m for s in streams for m in s], np.int32)
    offs = np.concatenate([[0], np.cumsum([len(s) for s in streams])]).astype(np.int64)
    compare(np.full(len(streams), cap, np.int32), msgs, offs, res, levels=2)


@pytest.mark.parametrize("res", ["regs", "tail", "tail_shallow", "lds", "unsorted"])
@pytest.mark.parametrize("cap", [2, 3])
def test_bruteforce_times_out_of_order(cap, res):
    """Random sequences of the small alphabet with times from a few values."""
    A = alphabet()
    rng = np.random.default_rng(900 + cap)
    seqs = [[A[j] for j in rng.integers(0, len(A), size=8)] for _ in range(4000)]
    times = rng.integers(0, 4, size=(len(seqs), 8))
    streams = [to_msgs(s, times=times[i]) for i, s in enumerate(seqs)]
    msgs = np.array([m for s in streams for m in s], np.int32)
    offs = np.concatenate([[0], np.cumsum([len(s) for s in streams])]).astype(np.int64)
    o = compare(np.full(len(streams), cap, np.int32), msgs, offs, res, levels=2)
    assert (o["stats"]["flags"] & lob.BOOK_TIME_ORDER).any()


@pytest.mark.parametrize("res", ["regs", "tail", "tail_shallow", "lds", "spill", "unsorted"])
@pytest.mark.parametrize("cap", [100, 300])
def test_flow_large_quantities(cap, res):
    if res == "tail" and cap > 128:
        pytest.skip("a capacity past 128 already runs the TAIL form")
    rng = np.random.default_rng(cap + 7)
    caps, msgs, offs = flow(rng, 24, 600, cap, big=True, shuffled_times=False)
    o = compare(caps, msgs, offs, res, levels=10)
    # the cases this test exists for did occur
    assert (o["trades"][:, 1].astype(np.int64) > (1 << 30)).any()
    assert (o["l2"][..., 1] == BIG).any()


@pytest.mark.parametrize("res", ["regs", "tail", "tail_shallow", "lds", "spill", "unsorted"])
@pytest.mark.parametrize("cap", [100, 300])
@pytest.mark.parametrize("l2", ["per_message", "final"])
@pytest.mark.parametrize("calls", [1, 3])
def test_flow_times_out_of_order(cap, res, l2, calls):
    """Per-message L2 or final L2 (the register kernel without a tail and without
    per-message L2 places such orders itself; its other forms hand the book to the
    LDS engine), in one call or three (later calls start with the book flagged)."""
    if res == "tail" and cap > 128:
        pytest.skip("a capacity past 128 already runs the TAIL form")
    rng = np.random.default_rng(cap + 11 + calls)
    caps, msgs, offs = flow(rng, 24, 600, cap, big=False, shuffled_times=True)
    mode = lob.L2_PER_MESSAGE if l2 == "per_message" else lob.L2_FINAL
    o = compare(caps, msgs, offs, res, levels=10, l2_mode=mode, calls=calls)
    assert (o["stats"]["flags"][:len(caps)] & lob.BOOK_TIME_ORDER).all()


def test_market_sweep_past_64_orders():
    """A market buy of INT32_MAX against 200 asks of 3e7 fills 71 of them whole and
    one in part (past the first 64-order chunk), in every residency; a second one
    fills 72 whole and one in part: 145 trades."""
    asks = [[1, -1, 10_000_000 + 100 * (k // 3), 30_000_000, k + 1, 2, 34200, k] for k in range(200)]
    mk = [[4, 1, 0, BIG, 1000, 9, 34201, 0], [4, 1, 0, BIG, 1001, 9, 34201, 1]]
    msgs = np.array(asks + mk, np.int32)
    offs = np.array([0, len(msgs)], np.int64)
    for res in ["regs", "lds", "spill", "unsorted"]:
        o = compare([250], msgs, offs, res, levels=10)
        assert np.diff(o["trade_offs"])[0] == 145
