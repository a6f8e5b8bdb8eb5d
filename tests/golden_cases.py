"""Parser for the hand-worked cases under tests/golden/ (format in its README)."""
import glob
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


class Case:
    def __init__(self, path):
        self.path = path
        self.name = os.path.splitext(os.path.basename(path))[0]
        self.cap = 4
        self.levels = 3
        self.msgs, self.trades, self.ask, self.bid = [], [], [], []
        self.l2ask = self.l2bid = None
        self.stats = {}
        self.cite = ""
        with open(path) as f:
            for raw in f:
                if raw.lstrip().startswith("# cite:"):
                    self.cite = raw.split(":", 1)[1].strip()
                line = raw.split("#", 1)[0].split()
                if not line:
                    continue
                key, vals = line[0], line[1:]
                if key == "cap":
                    self.cap = int(vals[0])
                elif key == "levels":
                    self.levels = int(vals[0])
                elif key == "msg":
                    assert len(vals) == 8, raw
                    self.msgs.append([int(v) for v in vals])
                elif key == "trade":
                    assert len(vals) == 7, raw
                    self.trades.append([int(v) for v in vals])
                elif key in ("ask", "bid"):
                    assert len(vals) == 6, raw
                    getattr(self, key).append([int(v) for v in vals])
                elif key in ("l2ask", "l2bid"):
                    setattr(self, key, np.array([int(v) for v in vals], np.int32).reshape(-1, 2))
                elif key == "stat":
                    self.stats[vals[0]] = int(vals[1])
                else:
                    raise ValueError(f"{path}: unknown line {raw!r}")
        assert self.cite, f"{path}: no citation"
        self.msgs = np.array(self.msgs, np.int32).reshape(-1, 8)
        self.trades = np.array(self.trades, np.int64).reshape(-1, 7)
        self.ask = np.array(self.ask, np.int32).reshape(-1, 6)
        self.bid = np.array(self.bid, np.int32).reshape(-1, 6)


def all_cases():
    return [Case(p) for p in sorted(glob.glob(os.path.join(GOLDEN, "*.txt")))]
