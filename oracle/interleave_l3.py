"""Explicit-state model checker for the third iceberg level's list protocol.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Operations that have reached level 3 (their primary and secondary buckets are
full without them) run find-or-put on one list of slabs, at the granularity
of the GPU kernel's steps:

* reading the list head, a slot of the current slab, or the slab's link is a
  separate step, and a plain read may return any value the location has held
  (a stale line in another XCD's cache): a slot EMPTY or its key, a head or
  link 0, the busy marker or the slab id;
* claiming a slot is one compare-and-swap from EMPTY; a lost claim adds the
  slot to the operation's known-occupied set and the slab is read again;
* setting a head or link is reserved by a compare-and-swap from 0 to BUSY;
  only the winner takes a slab from the pool (an atomic counter) and then
  publishes its id, or 0 and the answer FULL when the pool is used up;
* an operation that finds the location BUSY waits for it to change (its
  retries do not change any state, so waiting is the same as retrying).

At every terminal state the checker asserts: no BUSY left; the list is a
chain of distinct slabs and every slab taken from the pool is on it; in list
order the non-empty slots come first (every slab but the last is full); no
key is stored twice; one PUT per stored key and none for others; FOUND only
for stored keys; FULL only once the pool is used up.  A reachable cycle is
reported as non-termination, a state where unfinished operations cannot move
as a deadlock.
"""
from __future__ import annotations

from dataclasses import dataclass

EMPTY = 0
BUSY = -1
PUT, FOUND, FULL = "PUT", "FOUND", "FULL"


@dataclass
class L3Scenario:
    slots: int                 # key slots per slab (the link slot comes on top)
    pool: int                  # slabs in the pool
    keys: tuple                # one find-or-put per entry (repeats allowed)
    stale_reads: bool = True
    # planted mistakes (the checker must reject them)
    bug_alloc_first: bool = False   # take a slab before reserving the link (racing lanes take one each)
    bug_last_empty: bool = False    # claim the last empty slot instead of the first
    bug_skip_found: bool = False    # do not look for the key before claiming


# Memory: (head, links, cells, used, hist)
#   links[i], cells[i][j] for slab id i + 1; hist: frozenset of (location, value) ever held
# Operation: (phase, cur, known, snap, result, spare)


class L3Checker:
    def __init__(self, sc: L3Scenario):
        self.sc = sc
        self.errors: list[str] = []
        self.states = 0

    def initial(self):
        sc = self.sc
        hist = frozenset({("h", 0)} | {(("l", i + 1), 0) for i in range(sc.pool)})
        mem = (0, (0,) * sc.pool, ((EMPTY,) * sc.slots,) * sc.pool, 0, hist)
        ops = tuple(("H", 0, 0, (), None, 0) for _ in sc.keys)
        return (mem, ops)

    # -- memory helpers --------------------------------------------------------
    @staticmethod
    def _hist_add(hist, loc, v):
        return hist | {(loc, v)}

    def _read(self, mem, loc, current):
        """Values a plain read of `loc` may return."""
        if not self.sc.stale_reads:
            return {current}
        return {v for (l, v) in mem[4] if l == loc} | {current}

    def _set_link(self, mem, cur, v):
        head, links, cells, used, hist = mem
        if cur == 0:
            return (v, links, cells, used, self._hist_add(hist, "h", v))
        links = links[: cur - 1] + (v,) + links[cur:]
        return (head, links, cells, used, self._hist_add(hist, ("l", cur), v))

    def _get_link(self, mem, cur):
        return mem[0] if cur == 0 else mem[1][cur - 1]

    # -- moves -------------------------------------------------------------------
    def moves(self, state, t):
        sc = self.sc
        mem, ops = state
        head, links, cells, used, hist = mem
        phase, cur, known, snap, result, spare = ops[t]
        k = sc.keys[t]
        out = []

        def go(op, new_mem=None):
            new_ops = ops[:t] + (op,) + ops[t + 1:]
            out.append((new_mem if new_mem is not None else mem, new_ops))

        if phase == "done":
            return out
        if phase == "H":  # read the list head
            for v in self._read(mem, "h", head):
                if v in (0, BUSY):
                    go(("LK", 0, 0, (), None, spare))
                else:
                    go(("S", v, known, (), None, spare))
        elif phase == "LK":  # reserve the head (cur = 0) or the link of slab cur
            loc = self._get_link(mem, cur)
            if sc.bug_alloc_first and spare == 0:
                # take a slab first, then try to link it (the losing lanes keep theirs)
                if used < sc.pool:
                    go(("LK", cur, known, (), None, used + 1), (head, links, cells, used + 1, hist))
                else:
                    go(("done", cur, known, (), FULL, 0))
                return out
            if sc.bug_alloc_first:
                if loc == 0:
                    go(("S", spare, 0, (), None, 0), self._set_link(mem, cur, spare))
                elif loc != BUSY:
                    go(("S", loc, 0, (), None, spare))
                return out
            if loc == BUSY:
                return out  # waits until the reservation is resolved
            if loc == 0:
                go(("AL", cur, known, (), None, spare), self._set_link(mem, cur, BUSY))
            else:
                go(("S", loc, 0, (), None, spare))
        elif phase == "AL":  # take a slab from the pool (atomic counter)
            if used < sc.pool:
                go(("PB", cur, known, (), None, used + 1), (head, links, cells, used + 1, hist))
            else:
                go(("PB", cur, known, (), None, 0))
        elif phase == "PB":  # publish the slab, or release the reservation and answer FULL
            if spare:
                go(("S", spare, 0, (), None, 0), self._set_link(mem, cur, spare))
            else:
                go(("done", cur, known, (), FULL, 0), self._set_link(mem, cur, 0))
        elif phase == "S":  # read slot len(snap) of slab cur
            j = len(snap)
            cell = cells[cur - 1][j]
            vals = {cell, EMPTY} if sc.stale_reads else {cell}
            for v in vals:
                nsnap = snap + (v,)
                go(("S" if j + 1 < sc.slots else "D", cur, known, nsnap, None, spare))
        elif phase == "D":  # read the link with the slots and decide
            loc = self._get_link(mem, cur)
            for lv in self._read(mem, ("l", cur), loc):
                if not sc.bug_skip_found and k in snap:
                    go(("done", cur, known, (), FOUND, spare))
                    continue
                empties = [j for j, v in enumerate(snap) if v == EMPTY and not (known >> j) & 1]
                if empties:
                    j = empties[-1] if sc.bug_last_empty else empties[0]
                    go(("C", cur, known, (j,), None, spare))
                elif lv in (0, BUSY):
                    go(("LK", cur, known, (), None, spare))
                else:
                    go(("S", lv, 0, (), None, spare))
        elif phase == "C":  # CAS the chosen slot from EMPTY to k
            j = snap[0]
            cell = cells[cur - 1][j]
            if cell == EMPTY:
                row = cells[cur - 1][:j] + (k,) + cells[cur - 1][j + 1:]
                ncells = cells[: cur - 1] + (row,) + cells[cur:]
                go(("done", cur, known, (), PUT, spare), (head, links, ncells, used, hist))
            elif cell == k:
                go(("done", cur, known, (), FOUND, spare))
            else:
                go(("S", cur, known | (1 << j), (), None, spare))
        return out

    def _successors(self, state):
        out = []
        for t in range(len(self.sc.keys)):
            out.extend(self.moves(state, t))
        return out

    # -- checks ----------------------------------------------------------------
    def _check_terminal(self, state):
        sc = self.sc
        (head, links, cells, used, _), ops = state
        if head == BUSY or BUSY in links:
            return "a reservation was left BUSY"
        chain, seen, cur = [], set(), head
        while cur:
            if cur in seen or cur > used:
                return f"list is not a chain of taken slabs (slab {cur})"
            seen.add(cur)
            chain.append(cur)
            cur = links[cur - 1]
        if len(chain) != used:
            return f"{used - len(chain)} slab(s) taken from the pool are on no list"
        flat = [v for c in chain for v in cells[c - 1]]
        for i in range(1, len(flat)):
            if flat[i] != EMPTY and flat[i - 1] == EMPTY:
                return "a slot is filled after an empty slot in list order"
        stored = [v for v in flat if v != EMPTY]
        if len(stored) != len(set(stored)):
            return "a key is stored twice"
        for key in set(sc.keys):
            res = [ops[t][4] for t in range(len(sc.keys)) if sc.keys[t] == key]
            if key in stored and res.count(PUT) != 1:
                return f"key {key} is stored but {res.count(PUT)} operations answered PUT"
            if key not in stored and (PUT in res or FOUND in res):
                return f"key {key} is absent but an operation answered PUT or FOUND"
            if FULL in res and used < sc.pool:
                return f"key {key} answered FULL with {sc.pool - used} slab(s) left"
        return None

    def run(self, limit: int = 3_000_000):
        """Depth-first search over all interleavings; returns True if no
        error was found (errors are collected in self.errors)."""
        init = self.initial()
        color = {init: 1}
        stack = [(init, iter(self._successors(init)))]
        while stack and not self.errors:
            state, it = stack[-1]
            nxt = next(it, None)
            if nxt is None:
                color[state] = 2
                stack.pop()
                continue
            c = color.get(nxt, 0)
            if c == 1:
                self.errors.append("non-termination: a cycle of moves")
                break
            if c == 2:
                continue
            color[nxt] = 1
            self.states += 1
            if self.states > limit:
                self.errors.append("state limit reached")
                break
            succ = self._successors(nxt)
            if not succ:
                ops = nxt[1]
                if any(op[0] != "done" for op in ops):
                    self.errors.append("deadlock: unfinished operations cannot move")
                else:
                    err = self._check_terminal(nxt)
                    if err:
                        self.errors.append(err)
            stack.append((nxt, iter(succ)))
        return not self.errors


def check(sc: L3Scenario, limit: int = 3_000_000):
    c = L3Checker(sc)
    ok = c.run(limit)
    return ok, c.errors, c.states
