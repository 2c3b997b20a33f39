"""Explicit-state model checker for concurrent iceberg find-or-put.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Explores every interleaving of a few concurrent find-or-put operations on a
tiny abstract two-level table, at the granularity of the GPU kernel's steps:
each slot of a bucket snapshot is a separate read, a claim is one atomic
compare-and-swap, and a 16-bit slot claim is the compare-and-swap of the
32-bit word holding two slots, retried while only the neighbour half changed.
Reads model non-coherent caches: a read may return the slot's current value
or EMPTY (a stale line), since slots are written once.  Each operation keeps
known-occupied masks of slots where its claim failed, as the kernel does.

At every terminal state the checker asserts Theorem 1 (a)-(e) of Appendix A
and its corollary: the table is well-formed (the order property of
Definition 2 for every stored key, no key stored twice), every operation
returned FOUND, PUT or FULL, FOUND or PUT holds iff the key is in the table,
PUT holds iff that operation's claim stored the key, FULL implies the key's
three buckets are full without it, and at most one operation per key returns
PUT.  A reachable cycle (an operation that can run forever) is reported as
non-termination (Lemma 4).

Keys are abstract: a scenario gives each key its primary bucket and its two
secondary buckets, and the stored forms r'_0(k), (r_1(k), 0), (r_2(k), 1) are
the tuples (k, 0), (k, 1), (k, 2).
"""
from __future__ import annotations

import sys
from dataclasses import dataclass, field

EMPTY = None
PUT, FOUND, FULL = "PUT", "FOUND", "FULL"


@dataclass
class Scenario:
    B0: int                       # slots per primary bucket
    B1: int                       # slots per secondary bucket
    n_primary: int
    n_secondary: int
    ops: list                     # per operation: (key, primary bucket, secondary bucket 1, secondary bucket 2)
    prefill: dict = field(default_factory=dict)   # slot index -> stored form
    half_words: bool = False      # primary slots 2i, 2i+1 share one CAS word (16-bit slots)
    stale_reads: bool = True
    # planted mistakes (the checker must reject them)
    bug_no_known: bool = False    # forget failed claims (livelock under stale reads)
    bug_last_empty: bool = False  # claim the last instead of the first empty slot
    bug_skip_found2: bool = False  # no FOUND check on the secondary level
    bug_tie_to_1: bool = False     # pick secondary bucket 1 on ties (still correct: a consistent order)


def _slot(sc: Scenario, level: int, bucket: int, y: int) -> int:
    if level == 0:
        return bucket * sc.B0 + y
    return sc.n_primary * sc.B0 + bucket * sc.B1 + y


def _order(sc: Scenario):
    """Slot identities (x, y) of Definition 1 in increasing order."""
    ids = [(0, y) for y in range(sc.B0)]
    sec = []
    for y in range(sc.B1):
        if sc.bug_tie_to_1:
            sec += [(1, y), (2, y)]
        else:
            sec += [(2, y), (1, y)]
    return ids + sec


# Thread (operation) state: (phase, snapshot tuple, known0, known1, known2, aux, result, put_done)
#   phase: ("r1", i) reading primary slot i; ("c1", j) claim primary slot j;
#          ("w1", j, nb) 16-bit word claim with expected neighbour nb;
#          ("r2", i) reading secondary slot i of the 2*B1 (bucket 1 then 2);
#          ("c2", pick, j) claim secondary; ("done",)


class Checker:
    def __init__(self, sc: Scenario):
        self.sc = sc
        self.n_slots = sc.n_primary * sc.B0 + sc.n_secondary * sc.B1
        self.order = _order(sc)
        self.visited: set = set()
        self.on_stack: set = set()
        self.terminal = 0
        self.states = 0
        self.errors: list[str] = []

    # -- helpers -----------------------------------------------------------
    def _phys(self, op, x, y):
        k, p, s1, s2 = op
        if x == 0:
            return _slot(self.sc, 0, p, y)
        return _slot(self.sc, 1, s1 if x == 1 else s2, y)

    def _stored(self, op, x):
        return (op[0], x)

    def initial(self):
        table = [EMPTY] * self.n_slots
        for i, v in self.sc.prefill.items():
            table[i] = v
        threads = tuple((("r1", 0), (), 0, 0, 0, None, None) for _ in self.sc.ops)
        return (tuple(table), threads)

    def _reads(self, table, slot):
        v = table[slot]
        if v is EMPTY or not self.sc.stale_reads:
            return [v]
        return [v, EMPTY]

    # -- transitions of one operation ---------------------------------------
    def moves(self, state, t):
        """All successor states when operation t takes one step."""
        table, threads = state
        phase, snap, k0, k1, k2, res, put = threads[t]
        op = self.sc.ops[t]
        sc = self.sc
        out = []

        def with_thread(new_thread, new_table=None):
            th = list(threads)
            th[t] = new_thread
            return (table if new_table is None else new_table, tuple(th))

        if phase[0] == "r1":
            i = phase[1]
            for v in self._reads(table, self._phys(op, 0, i)):
                s2 = snap + (v,)
                if i + 1 < sc.B0:
                    out.append(with_thread((("r1", i + 1), s2, k0, k1, k2, res, put)))
                else:
                    out.append(with_thread(self._decide1(op, s2, k0, k1, k2, put)))
            return out
        if phase[0] == "c1":
            j = phase[1]
            slot = self._phys(op, 0, j)
            e = self._stored(op, 0)
            if sc.half_words:
                nb_y = j ^ 1
                nb = snap[nb_y] if nb_y < len(snap) else EMPTY
                return [with_thread((("w1", j, nb), snap, k0, k1, k2, res, put))]
            cur = table[slot]
            if cur is EMPTY:
                tb = list(table)
                tb[slot] = e
                return [with_thread((("done",), (), k0, k1, k2, PUT, True), tuple(tb))]
            if cur == e:
                return [with_thread((("done",), (), k0, k1, k2, FOUND, put))]
            nk0 = k0 if sc.bug_no_known else (k0 | (1 << j))
            return [with_thread((("r1", 0), (), nk0, k1, k2, res, put))]
        if phase[0] == "w1":
            j, nb = phase[1], phase[2]
            slot = self._phys(op, 0, j)
            nbslot = self._phys(op, 0, j ^ 1)
            e = self._stored(op, 0)
            cur, curnb = table[slot], table[nbslot]
            if cur is EMPTY and curnb == nb:  # word compares equal: store
                tb = list(table)
                tb[slot] = e
                return [with_thread((("done",), (), k0, k1, k2, PUT, True), tuple(tb))]
            if cur is not EMPTY:
                if cur == e:
                    return [with_thread((("done",), (), k0, k1, k2, FOUND, put))]
                nk0 = k0 if sc.bug_no_known else (k0 | (1 << j))
                return [with_thread((("r1", 0), (), nk0, k1, k2, res, put))]
            # only the neighbour half differed: retry with the value found
            return [with_thread((("w1", j, curnb), snap, k0, k1, k2, res, put))]
        if phase[0] == "r2":
            i = phase[1]
            x = 1 if i < sc.B1 else 2
            y = i % sc.B1
            for v in self._reads(table, self._phys(op, x, y)):
                s2 = snap + (v,)
                if i + 1 < 2 * sc.B1:
                    out.append(with_thread((("r2", i + 1), s2, k0, k1, k2, res, put)))
                else:
                    out.append(with_thread(self._decide2(op, s2, k0, k1, k2, put)))
            return out
        if phase[0] == "c2":
            x, j = phase[1], phase[2]
            slot = self._phys(op, x, j)
            e = self._stored(op, x)
            cur = table[slot]
            if cur is EMPTY:
                tb = list(table)
                tb[slot] = e
                return [with_thread((("done",), (), k0, k1, k2, PUT, True), tuple(tb))]
            if cur == e:
                return [with_thread((("done",), (), k0, k1, k2, FOUND, put))]
            if sc.bug_no_known:
                return [with_thread((("r2", 0), (), k0, k1, k2, res, put))]
            if x == 1:
                return [with_thread((("r2", 0), (), k0, k1 | (1 << j), k2, res, put))]
            return [with_thread((("r2", 0), (), k0, k1, k2 | (1 << j), res, put))]
        return out

    def _decide1(self, op, snap, k0, k1, k2, put):
        e = self._stored(op, 0)
        if any(v == e for v in snap):
            return (("done",), (), k0, k1, k2, FOUND, put)
        empties = [y for y in range(self.sc.B0) if snap[y] is EMPTY and not (k0 >> y) & 1]
        if not empties:
            return (("r2", 0), (), k0, k1, k2, None, put)
        j = empties[-1] if self.sc.bug_last_empty else empties[0]
        return (("c1", j), snap, k0, k1, k2, None, put)

    def _decide2(self, op, snap, k0, k1, k2, put):
        B1 = self.sc.B1
        b1, b2 = snap[:B1], snap[B1:]
        if not self.sc.bug_skip_found2:
            if any(v == self._stored(op, 1) for v in b1) or any(v == self._stored(op, 2) for v in b2):
                return (("done",), (), k0, k1, k2, FOUND, put)
        e1 = [y for y in range(B1) if b1[y] is EMPTY and not (k1 >> y) & 1]
        e2 = [y for y in range(B1) if b2[y] is EMPTY and not (k2 >> y) & 1]
        l1 = e1[0] if e1 else B1
        l2 = e2[0] if e2 else B1
        pick1 = (l1 <= l2) if self.sc.bug_tie_to_1 else (l1 < l2)
        lp = l1 if pick1 else l2
        if lp == B1:
            return (("done",), (), k0, k1, k2, FULL, put)
        return (("c2", 1 if pick1 else 2, lp), snap, k0, k1, k2, None, put)

    # -- exploration -------------------------------------------------------
    def run(self, limit: int = 2_000_000):
        sys.setrecursionlimit(100000)
        start = self.initial()
        stack = [(start, iter(self._successors(start)))]
        self.on_stack.add(start)
        self.visited.add(start)
        while stack and not self.errors:
            state, it = stack[-1]
            nxt = next(it, None)
            if nxt is None:
                stack.pop()
                self.on_stack.discard(state)
                continue
            if nxt in self.on_stack:
                self.errors.append("non-termination: a cycle of steps is reachable")
                break
            if nxt in self.visited:
                continue
            self.visited.add(nxt)
            self.states += 1
            if self.states > limit:
                self.errors.append("state limit exceeded")
                break
            succ = self._successors(nxt)
            if not succ:
                self.terminal += 1
                self._check_terminal(nxt)
                continue
            self.on_stack.add(nxt)
            stack.append((nxt, iter(succ)))
        return not self.errors

    def _successors(self, state):
        out = []
        for t in range(len(self.sc.ops)):
            if state[1][t][0][0] != "done":
                out.extend(self.moves(state, t))
        return out

    def _check_terminal(self, state):
        table, threads = state
        sc = self.sc
        # (a) well-formed: order property and no duplicates
        where = {}
        for op in sc.ops:
            k = op[0]
            for x, y in self.order:
                if table[self._phys(op, x, y)] == (k, x):
                    where.setdefault(k, set()).add((x, y))
        for k, locs in where.items():
            if len(locs) > 1:
                self.errors.append(f"key {k} stored twice: {sorted(locs)}")
                return
            (x, y), = locs
            op = next(o for o in sc.ops if o[0] == k)
            for xx, yy in self.order:
                if (xx, yy) == (x, y):
                    break
                v = table[self._phys(op, xx, yy)]
                if v is EMPTY:
                    self.errors.append(f"order property: {k} at {(x, y)}, earlier slot {(xx, yy)} empty")
                    return
        present = set(where)
        puts = {}
        for t, op in enumerate(sc.ops):
            k = op[0]
            res, put = threads[t][5], threads[t][6]
            if res not in (PUT, FOUND, FULL):
                self.errors.append(f"operation {t} ended without a result")
                return
            if (res in (PUT, FOUND)) != (k in present):
                self.errors.append(f"operation {t} on {k}: {res} but key present={k in present}")
                return
            if (res == PUT) != bool(put):
                self.errors.append(f"operation {t}: result {res} but stored={put}")
                return
            if res == PUT:
                puts[k] = puts.get(k, 0) + 1
            if res == FULL:
                for x, y in self.order:
                    v = table[self._phys(op, x, y)]
                    if v is EMPTY or v == (k, x):
                        self.errors.append(f"operation {t} FULL but slot {(x, y)} is {v}")
                        return
        for k, n in puts.items():
            if n > 1:
                self.errors.append(f"key {k} PUT {n} times")
                return


def check(sc: Scenario, limit: int = 2_000_000):
    c = Checker(sc)
    ok = c.run(limit)
    return ok, c.errors, c.states, c.terminal
