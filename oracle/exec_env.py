"""Execution environment of JAX-LOB (Frey et al. 2023), Section 5.2, on the oracle
engine -- TEST INFRASTRUCTURE ONLY: the tests use it; the product path never
imports it.

Plain and step by step, one book at a time:
  1. the action (order sizes at the far-touch, mid, near-touch and passive prices,
     Section 5.2.3) becomes agent limit orders priced off the book as it stands;
     from one minute before the episode end a market order for the remaining task
     quantity replaces them (Section 5.2.5);
  2. the step's data messages, then the agent orders, go through the engine; the
     level-1 state is read after every data message (Section 5.2.1);
  3. the observation (Section 5.2.2) and the reward of eqs. (rewardfunc) and (vwap),
     Section 5.2.4, are formed from those level-1 rows and the step's trades.

Readings (the paper leaves these open): R15 the mid price is floor((ask + bid) / 2)
in price units and a missing best price reads -1 (mid, passive and spread then read
-1 too, a missing side's quantity reads 0); R16 agent orders carry the time of the
step's last data message and consecutive ids; R17 Q_j is capped so that the
executed quantity never exceeds the task size, and a step without trades has
reward 0; R18 the drift uses the mid price after the step's last data message (0 if
missing); the episode is over once the current time reaches end_s.
"""
import numpy as np

from . import oracle as O


class ExecEnv:
    def __init__(self, book, task_side, task_qty, p_init, start, end_s, next_oid, tick=100, passive_ticks=1,
                 agent_tid=-1, lam=0.0):
        self.book = book
        self.side = 1 if task_side == 1 else -1
        self.task_qty = int(task_qty)
        self.exec_qty = 0
        self.revenue = 0
        self.done = 0
        self.p_init = int(p_init)
        self.start = (int(start[0]), int(start[1]))
        self.end_s = int(end_s)
        self.next_oid = int(next_oid)
        self.tick = int(tick)
        self.n = int(passive_ticks)
        self.tid = int(agent_tid)
        self.lam = float(lam)
        self.last_time = (0, 0)

    def _best(self):
        a, b = self.book.dump(0), self.book.dump(1)
        return (int(a[0, 0]) if len(a) else -1), (int(b[0, 0]) if len(b) else -1)

    def _prices(self, ask, bid):
        """far touch, mid, near touch, passive (Section 5.2.2 and 5.2.3; R15)"""
        buy = self.side == 1
        far = ask if buy else bid
        near = bid if buy else ask
        mid = (ask + bid) // 2 if ask >= 0 and bid >= 0 else -1
        if near < 0:
            passive = -1
        else:
            passive = near - self.n * self.tick if buy else near + self.n * self.tick
            if passive <= 0:
                passive = -1
        return far, mid, near, passive

    def step(self, window, action_qty):
        window = np.asarray(window, np.int32)
        valid = [m for m in window if 1 <= m[0] <= 4]
        t = (int(valid[-1][6]), int(valid[-1][7])) if valid else self.last_time
        # 1. the agent's orders (R16)
        orders = []
        remaining = self.task_qty - self.exec_qty
        if not self.done and remaining > 0:
            if t[0] >= self.end_s - 60:
                orders.append([4, self.side, 0, remaining, self.next_oid, self.tid, t[0], t[1]])
                self.next_oid += 1
            else:
                ask, bid = self._best()
                for q, px in zip(action_qty, self._prices(ask, bid)):
                    if q > 0 and px > 0:
                        orders.append([1, self.side, px, int(q), self.next_oid, self.tid, t[0], t[1]])
                        self.next_oid += 1
        # 2. data messages with the level-1 state after each, then the agent's orders
        trades = []
        l1 = []
        for m in window:
            trades.extend(self.book.process(m))
            if 1 <= m[0] <= 4:
                self.last_time = (int(m[6]), int(m[7]))
            l1.append(self.book.l2(1).reshape(-1))  # ask P, ask Q, bid P, bid Q
        for m in orders:
            trades.extend(self.book.process(np.array(m, np.int32)))
            self.last_time = (int(m[6]), int(m[7]))
        # 3. observation
        W = len(window)
        obs = np.zeros(6 * W + 8, np.int64)
        mids = []
        for k, (ap, aq, bp, bq) in enumerate(l1):
            ask = int(ap) if aq > 0 else -1
            bid = int(bp) if bq > 0 else -1
            mid = (ask + bid) // 2 if ask >= 0 and bid >= 0 else -1
            near = ask if self.side == -1 else bid
            if near < 0:
                passive = -1
            else:
                passive = near + self.n * self.tick if self.side == -1 else near - self.n * self.tick
                if passive <= 0:
                    passive = -1
            obs[k] = bid
            obs[W + k] = ask
            obs[2 * W + k] = mid
            obs[3 * W + k] = passive
            obs[4 * W + k] = ask - bid if ask >= 0 and bid >= 0 else -1
            obs[5 * W + k] = (int(aq) if aq > 0 else 0) - (int(bq) if bq > 0 else 0)
            mids.append(mid)
        # reward (eqs. rewardfunc, vwap; R17)
        fills = [tr for tr in trades if tr[6] == self.tid or tr[7] == self.tid]
        A = B = 0
        for tr in fills:
            take = min(int(tr[1]), self.task_qty - self.exec_qty - B)
            if take <= 0:
                continue
            A += take * int(tr[0])
            B += take
        S_QP = sum(int(tr[0]) * int(tr[1]) for tr in trades)
        S_Q = sum(int(tr[1]) for tr in trades)
        if S_Q > 0:
            vwap = np.float64(S_QP) / np.float64(S_Q)
            bv = np.float64(B) * vwap
            reward = (np.float64(A) - bv) + np.float64(self.lam) * (bv - np.float64(B) * np.float64(self.p_init))
        else:
            reward = np.float64(0.0)
        self.exec_qty += B
        self.revenue += A
        el = [t[0] - self.start[0], t[1] - self.start[1]]
        if el[1] < 0:
            el = [el[0] - 1, el[1] + 1_000_000_000]
        last_mid = mids[-1] if mids else -1
        obs[6 * W:] = [t[0], t[1], el[0], el[1], self.p_init, last_mid - self.p_init if last_mid >= 0 else 0,
                       self.task_qty, self.exec_qty]
        self.done = 1 if (self.exec_qty >= self.task_qty or t[0] >= self.end_s) else 0
        fills6 = np.array([tr[:6] for tr in fills], np.int32).reshape(-1, 6)
        return obs.astype(np.int32), float(reward), fills6


def new_book(cap):
    return O.Book(cap)
