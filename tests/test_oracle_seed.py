"""Oracle book initialisation from an L2 snapshot (JAX-LOB Section 5.1.1; reading
R14): pinned by a hand-worked example, by the snapshot round trip (seed, then L2,
gives the snapshot back), by refusal of snapshots that are not books, and by the
initial-order cancel rule acting on seeded orders."""
import numpy as np
import pytest

from oracle import oracle as O


def snap(asks, bids, levels):
    """[2][levels][2] from lists of (price, qty), missing levels (-1, 0)."""
    out = np.zeros((2, levels, 2), np.int32)
    out[:, :, 0] = -1
    for sd, lv in enumerate((asks, bids)):
        for k, (p, q) in enumerate(lv):
            out[sd, k] = (p, q)
    return out


def test_hand_worked_ids_and_fields():
    # two ask levels, three bid levels: ids go level by level, ask before bid
    b = O.Book(5)
    n = b.seed_l2(snap([(101, 5), (102, 7)], [(99, 3), (98, 4), (97, 1)], 3), tid=4, ts=34200, tns=17)
    assert n == 5
    np.testing.assert_array_equal(b.dump(0), [[101, 5, -9000, 4, 34200, 17], [102, 7, -9002, 4, 34200, 17]])
    np.testing.assert_array_equal(b.dump(1), [[99, 3, -9001, 4, 34200, 17], [98, 4, -9003, 4, 34200, 17],
                                              [97, 1, -9004, 4, 34200, 17]])
    st = b.stats()
    assert st["n_msgs"] == 0 and st["limit_qty"] == 0 and st["flags"] == 0


def test_missing_levels_skipped_in_id_order():
    # a one-sided book: only bids; the ids stay consecutive
    b = O.Book(4)
    assert b.seed_l2(snap([], [(50, 2), (40, 9)], 4)) == 2
    np.testing.assert_array_equal(b.dump(1)[:, 2], [-9000, -9001])
    assert len(b.dump(0)) == 0


@pytest.mark.parametrize("seed", range(6))
def test_round_trip_of_a_replayed_book(seed):
    """Any book the engine produces: seeding a second book from its L2 gives an L2
    equal to the snapshot (one order per level, the level's quantity)."""
    rng = np.random.default_rng(seed)
    a = O.Book(64)
    t = 0
    for k in range(400):
        side = 1 if rng.random() < 0.5 else -1
        mid = 1000
        px = mid + int(rng.integers(-8, 9))
        typ = 1 if rng.random() < 0.8 else 4
        a.process([typ, side, px, int(rng.integers(1, 30)), k + 1, 1, 34200, t])
        t += 1
    levels = 10
    s = a.l2(levels)
    b = O.Book(64)
    n = b.seed_l2(s, tid=9, ts=34300, tns=0)
    assert n == int((s[:, :, 1] > 0).sum())
    np.testing.assert_array_equal(b.l2(levels), s)
    # the seeded book has exactly one order per price level
    for sd in (0, 1):
        d = b.dump(sd)
        assert len(np.unique(d[:, 0])) == len(d)


@pytest.mark.parametrize("asks,bids,cap", [
    ([(101, 5)], [(101, 3)], 4),              # crossed (bid == ask)
    ([(101, 5)], [(105, 3)], 4),              # crossed
    ([(102, 5), (101, 1)], [(99, 3)], 4),     # asks not ascending
    ([(101, 5)], [(97, 3), (99, 1)], 4),      # bids not descending
    ([(101, 5), (101, 2)], [(99, 3)], 4),     # repeated price
    ([(101, 1), (102, 1), (103, 1)], [], 2),  # more levels than capacity
])
def test_not_a_book_is_refused(asks, bids, cap):
    b = O.Book(cap)
    b.process([1, 1, 50, 5, 1, 1, 1, 0])  # something to be cleared
    assert b.seed_l2(snap(asks, bids, 4)) == -1
    assert b.stats()["flags"] & O.FLAG_BAD_LOAD
    assert len(b.dump(0)) == 0 and len(b.dump(1)) == 0


def test_seeded_orders_take_the_initial_order_cancel_rule():
    """Section 5.1.1: a cancel whose id is unknown but whose price matches a seeded
    (id <= -9000) order reduces that order."""
    b = O.Book(8)
    b.seed_l2(snap([(101, 5), (102, 7)], [(99, 3)], 2), ts=34200)
    b.process([2, -1, 102, 4, 555, 1, 34201, 0])   # unknown id 555 at the second ask level
    np.testing.assert_array_equal(b.dump(0)[:, :3], [[101, 5, -9000], [102, 3, -9002]])
    b.process([3, 1, 99, 3, 556, 1, 34201, 1])     # delete the whole bid level
    assert len(b.dump(1)) == 0
    assert b.stats()["cancel_miss"] == 0 and b.stats()["cancelled_qty"] == 7


def test_seed_time_is_the_books_latest_time():
    """R14: the initial orders' time is the book's latest time.  A message stamped
    before it is flagged as time going backwards, and at an equal price it ranks
    ahead of the seeded order (Section 4.1: earliest time first); one stamped at
    it leaves the book unflagged and ranks behind (equal times: arrival order)."""
    b = O.Book(8)
    b.seed_l2(snap([(101, 5)], [(99, 3)], 2), tid=4, ts=34200, tns=17)
    b.process([1, 1, 99, 2, 1, 1, 34200, 17])
    assert b.stats()["flags"] == 0
    np.testing.assert_array_equal(b.dump(1)[:, 2], [-9001, 1])
    b = O.Book(8)
    b.seed_l2(snap([(101, 5)], [(99, 3)], 2), tid=4, ts=34200, tns=17)
    b.process([1, 1, 99, 6, 2, 1, 34200, 16])
    assert b.stats()["flags"] & O.FLAG_TIME_ORDER
    np.testing.assert_array_equal(b.dump(1)[:, 2], [2, -9001])
    np.testing.assert_array_equal(b.l2(1)[1], [[99, 9]])
