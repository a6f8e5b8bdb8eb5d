"""Windowed replay data (lob_windows; JAX-LOB Section 5.1.1, data loading), host
code of liblob, against a plain Python split of the same stream."""
import numpy as np
import pytest

from paper_2308_13289_amd import lob
from paper_2308_13289_amd import workload as W


def stream(n_flow=4000, seed_tag=11):
    w = W.uniform(1, n_flow, cap=100, tag=seed_tag)
    return w.msgs


def plain_split(msgs, start_s, window_s, per_step, n_windows):
    out = []
    for k in range(n_windows):
        lo, hi = start_s + k * window_s, start_s + (k + 1) * window_s
        sel = np.nonzero((msgs[:, 6] >= lo) & (msgs[:, 6] < hi))[0]
        out.append(sel)
    return out


@pytest.mark.parametrize("start_s,window_s,per_step", [(34200, 1, 100), (34201, 2, 64), (34199, 1, 7)])
def test_windows_match_plain_split(start_s, window_s, per_step):
    msgs = stream()
    n_windows = 3
    ref = plain_split(msgs, start_s, window_s, per_step, n_windows)
    max_steps = max(-(-len(r) // per_step) for r in ref) + 2
    win, steps, first = lob.windows(msgs, start_s, window_s, per_step, max_steps, n_windows)
    assert win.shape == (n_windows, max_steps, per_step, 8)
    for k, sel in enumerate(ref):
        assert steps[k] == -(-len(sel) // per_step)
        if len(sel):
            assert first[k] == sel[0] and first[k + 1] >= sel[-1] + 1
        flat = win[k].reshape(-1, 8)
        np.testing.assert_array_equal(flat[:len(sel)], msgs[sel])
        assert (flat[len(sel):] == 0).all()  # padding: type 0, never processed
    assert (np.diff(first) >= 0).all()


def test_count_only_and_too_few_steps():
    msgs = stream()
    with pytest.raises(lob.LobError):
        lob.windows(msgs, 34200, 1, 100, 1, 2)
    steps = np.zeros(2, np.int32)
    first = np.zeros(3, np.int64)
    st = lob.load().lob_windows(msgs.ctypes.data, len(msgs), 34200, 1, 100, 0, 2, None, steps.ctypes.data,
                                first.ctypes.data)
    assert st == lob.ECAP and (steps == 0).all()  # max_steps 0: counted, nothing kept


def test_bad_arguments():
    msgs = stream(200)
    back = msgs.copy()
    back[-1, 6] = back[0, 6] - 5  # a time that jumps back across window boundaries
    with pytest.raises(lob.LobError):
        lob.windows(back, int(back[0, 6]) - 10, 1, 10, 100, 40)
    with pytest.raises(lob.LobError):
        lob.windows(msgs, 34200, 0, 10, 10, 1)
    win, steps, first = lob.windows(np.zeros((0, 8), np.int32), 0, 1, 4, 2, 2)
    assert (steps == 0).all() and (first == 0).all() and (win == 0).all()
