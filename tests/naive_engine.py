"""A second matching engine, written independently of the oracle, for brute-force
differential tests on tiny inputs.

Textbook formulation: a book side is a Python list of live orders that is
re-sorted into priority order (price, then time, then arrival) every time it is
looked at; a fill is min(remaining, resting).  It shares no code with the oracle
(which keeps unsorted fixed arrays and applies the paper's Q_s'/Q_a' update and
clean-up pass) and exists only for tests.
"""
INT32_MAX = 2 ** 31 - 1


class Order:
    __slots__ = ("price", "qty", "oid", "tid", "ts", "tns", "arrival")

    def __init__(self, price, qty, oid, tid, ts, tns, arrival):
        self.price, self.qty, self.oid, self.tid = price, qty, oid, tid
        self.ts, self.tns, self.arrival = ts, tns, arrival

    def row(self):
        return [self.price, self.qty, self.oid, self.tid, self.ts, self.tns]


class NaiveBook:
    def __init__(self, cap):
        self.cap = cap
        self.sides = {1: [], -1: []}  # +1 bids, -1 asks
        self.arrivals = 0
        self.rejected = self.cancelled = self.discarded = self.misses = 0

    def ranked(self, side):
        if side == 1:
            key = lambda o: (-o.price, o.ts, o.tns, o.arrival)
        else:
            key = lambda o: (o.price, o.ts, o.tns, o.arrival)
        return sorted(self.sides[side], key=key)

    def process(self, m):
        T, S, P, Q, OID, TID, Ts, Tns = (int(v) for v in m)
        if T not in (1, 2, 3, 4) or S not in (1, -1):
            return []
        if T in (2, 3):
            self._cancel(S, P, Q, OID)
            return []
        if T == 1:
            limit = P
        else:
            limit = INT32_MAX if S == 1 else 0
        left = Q
        out = []
        while left > 0:
            queue = self.ranked(-S)
            if not queue:
                break
            top = queue[0]
            crosses = top.price <= limit if S == 1 else top.price >= limit
            if not crosses:
                break
            fill = min(left, top.qty)
            out.append([top.price, fill, top.oid, OID, Ts, Tns, top.tid, TID])
            top.qty -= fill
            left -= fill
            if top.qty == 0:
                self.sides[-S].remove(top)
        if T == 1 and left > 0:
            if len(self.sides[S]) < self.cap:
                self.sides[S].append(Order(P, left, OID, TID, Ts, Tns, self.arrivals))
                self.arrivals += 1
            else:
                self.rejected += left
        elif T == 4 and left > 0:
            self.discarded += left
        return out

    def _cancel(self, S, P, Q, OID):
        if Q <= 0:
            return
        ranked = self.ranked(S)
        hit = [o for o in ranked if o.oid == OID]
        if not hit:
            hit = [o for o in ranked if o.oid <= -9000 and o.price == P]
        if not hit:
            self.misses += 1
            return
        o = hit[0]
        self.cancelled += min(Q, o.qty)
        o.qty -= Q
        if o.qty <= 0:
            self.sides[S].remove(o)

    def dump(self, side):
        return [o.row() for o in self.ranked(side)]

    def l2(self, levels):
        out = []
        for side in (-1, 1):
            agg = {}
            for o in self.sides[side]:
                agg[o.price] = agg.get(o.price, 0) + o.qty
            prices = sorted(agg, reverse=(side == 1))[:levels]
            # the L2 record is int32: a level's exact sum is reported capped at INT32_MAX
            rows = [[p, min(agg[p], INT32_MAX)] for p in prices] + [[-1, 0]] * (levels - len(prices))
            out.append(rows)
        return out
