"""Explicit-state model checker for the concurrent compact cuckoo put.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Explores every interleaving of a few concurrent cuckoo puts (Sec. 4.4,
Alg. 4) on a tiny abstract table, at the granularity of the GPU kernel's
steps.  An operation carries a key k with hash index j and round counter c:

* it reads the slots of bucket a_j(k) one at a time; a read may return the
  slot's current value or EMPTY (a stale line of a non-coherent cache: a
  slot, once written, is never EMPTY again, so staleness can only hide an
  occupant);
* if some slot read EMPTY and is not in the operation's known-occupied mask,
  it claims the first such slot (with claim_any: any such slot, every choice
  explored) with one compare-and-swap; a lost claim adds the slot to the mask
  and uses up the round;
* otherwise (every slot occupied) it swaps (r_j(k), j) into a victim row with
  one atomic exchange; the evicted word (r', j') together with the bucket
  address decodes, under permutation j', to the key k' that the operation
  carries on with hash index j' + 1 mod H and an empty mask;
* every round increments c; after C rounds the carried key is dropped and the
  answer is FULL.

Keys are abstract: a scenario lists, per key and hash index j, the bucket
a_j(k) and the remainder r_j(k); a slot stores (r, j), so decoding a slot
means finding the key with that bucket and remainder under permutation j.
Victim rows are explored exhaustively (the kernel picks them by hashing the
carried key and the round; correctness must not depend on the choice).

At every terminal state the checker asserts: every operation answered PUT or
FULL; every slot decodes to a key of the scenario, under its own tag, in the
bucket of that tag; no key is stored twice; the stored keys are the
pre-filled and put keys minus exactly one dropped key per FULL answer (no
key lost on eviction); a key stored under tag j > 0 has a full bucket
a_{j-1} (the invariant behind the lookup's early exit); the sequential
lookup (buckets a_0, a_1, ... up to the first that is not full) finds
exactly the stored keys; and, where the scenario leaves room, no FULL.  A
reachable cycle would be non-termination.
"""
from __future__ import annotations

import sys
from dataclasses import dataclass, field

EMPTY = None
PUT, FULL = "PUT", "FULL"


@dataclass
class CuckooScenario:
    B: int                        # slots per bucket
    n_buckets: int
    H: int                        # hash functions
    C: int                        # chain bound (rounds)
    keys: dict                    # key -> tuple over j of (bucket a_j, remainder r_j)
    ops: list                     # keys put concurrently (distinct, not pre-filled)
    prefill: dict = field(default_factory=dict)   # slot index -> key stored there under tag (slot's value)
    prefill_tags: dict = field(default_factory=dict)  # slot index -> tag j of the pre-filled key
    stale_reads: bool = True
    expect_no_full: bool = False  # the table has room and C is large enough: every put must succeed
    # claim any free slot of the snapshot (every choice explored) instead of
    # the first: Alg. 4 asks only for some empty slot, and the kernel spreads
    # the claims of keys that contend for one bucket over its empty slots
    claim_any: bool = False
    # planted mistakes (the checker must reject them)
    bug_decode_with_carried_j: bool = False  # decode the evicted word with the carried key's j
    bug_no_known: bool = False               # forget lost claims


class CuckooChecker:
    def __init__(self, sc: CuckooScenario):
        self.sc = sc
        self.n_slots = sc.n_buckets * sc.B
        self.decode = {}
        for k, per in sc.keys.items():
            assert len(per) == sc.H
            for j, (a, r) in enumerate(per):
                assert (j, a, r) not in self.decode, "pi_j must be a bijection: (bucket, remainder) repeats"
                self.decode[(j, a, r)] = k
        self.visited: set = set()
        self.on_stack: set = set()
        self.states = 0
        self.terminal = 0
        self.errors: list[str] = []

    # -- table encoding ------------------------------------------------------
    def _bucket_of(self, k, j):
        if isinstance(k, tuple):  # a key that decoding made up (only under a planted mistake)
            return k[1]
        return self.sc.keys[k][j][0]

    def _form(self, k, j):
        """The slot word of key k under hash j: (remainder, tag)."""
        if isinstance(k, tuple):
            return (k[2], j)
        return (self.sc.keys[k][j][1], j)

    def _decode(self, bucket, word, j_used):
        r, _tag = word
        k = self.decode.get((j_used, bucket, r))
        return k if k is not None else ("?", bucket, r)  # no such key: a made-up one

    def initial(self):
        table = [EMPTY] * self.n_slots
        for slot, k in self.sc.prefill.items():
            j = self.sc.prefill_tags.get(slot, 0)
            assert slot // self.sc.B == self._bucket_of(k, j), "pre-filled key outside its bucket"
            table[slot] = self._form(k, j)
        # thread: (phase, carried key, j, c, known, snapshot, result)
        threads = tuple((("r", 0), k, 0, 1, 0, (), None) for k in self.sc.ops)
        return (tuple(table), threads)

    def _reads(self, v):
        if v is EMPTY or not self.sc.stale_reads:
            return [v]
        return [v, EMPTY]

    # -- one step of operation t --------------------------------------------
    def moves(self, state, t):
        table, threads = state
        phase, k, j, c, known, snap, res = threads[t]
        sc = self.sc
        a = self._bucket_of(k, j)

        def th(new, tb=None):
            ts = list(threads)
            ts[t] = new
            return (table if tb is None else tb, tuple(ts))

        def next_round(k2, j2, known2):
            if c + 1 > sc.C:
                return (("done",), k2, j2, c + 1, known2, (), FULL)
            return (("r", 0), k2, j2, c + 1, known2, (), None)

        if phase[0] == "r":
            i = phase[1]
            out = []
            for v in self._reads(table[a * sc.B + i]):
                s2 = snap + (v is EMPTY,)
                if i + 1 < sc.B:
                    out.append(th((("r", i + 1), k, j, c, known, s2, None)))
                else:
                    free = [y for y in range(sc.B) if s2[y] and not (known >> y) & 1]
                    if free:
                        for q in (free if sc.claim_any else free[:1]):
                            out.append(th((("claim", q), k, j, c, known, (), None)))
                    else:
                        out.append(th((("evict",), k, j, c, known, (), None)))
            return out
        if phase[0] == "claim":
            q = phase[1]
            slot = a * sc.B + q
            if table[slot] is EMPTY:
                tb = list(table)
                tb[slot] = self._form(k, j)
                return [th((("done",), k, j, c, known, (), PUT), tuple(tb))]
            known2 = known if sc.bug_no_known else known | (1 << q)
            return [th(next_round(k, j, known2))]
        if phase[0] == "evict":
            out = []
            for v in range(sc.B):  # every victim row
                slot = a * sc.B + v
                old = table[slot]
                tb = list(table)
                tb[slot] = self._form(k, j)
                tb = tuple(tb)
                if old is EMPTY:  # cannot happen: eviction only follows a full snapshot
                    out.append((tb, threads[:t] + ((("done",), k, j, c, known, (), PUT),) + threads[t + 1:]))
                    continue
                j_old = old[1]
                k2 = self._decode(a, old, j if sc.bug_decode_with_carried_j else j_old)
                j2 = (j_old + 1) % sc.H
                ts = list(threads)
                ts[t] = next_round(k2, j2, 0)
                out.append((tb, tuple(ts)))
            return out
        return []

    # -- exploration -----------------------------------------------------------
    def _successors(self, state):
        out = []
        for t in range(len(self.sc.ops)):
            if state[1][t][0][0] != "done":
                out.extend(self.moves(state, t))
        return out

    def run(self, limit: int = 3_000_000):
        sys.setrecursionlimit(100000)
        start = self.initial()
        stack = [(start, iter(self._successors(start)))]
        self.visited.add(start)
        self.on_stack.add(start)
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

    def _lookup(self, table, k):
        """Sequential lookup (Sec. 4.4): buckets a_0, a_1, ... in order; a hit
        answers 1, a bucket that is not full and lacks k answers 0."""
        sc = self.sc
        for j in range(sc.H):
            a = self._bucket_of(k, j)
            words = table[a * sc.B:(a + 1) * sc.B]
            if self._form(k, j) in words:
                return 1
            if any(w is EMPTY for w in words):
                return 0
        return 0

    def _check_terminal(self, state):
        table, threads = state
        sc = self.sc
        results = [th[6] for th in threads]
        if any(r not in (PUT, FULL) for r in results):
            self.errors.append(f"an operation ended without PUT or FULL: {results}")
            return
        stored = []
        for slot, w in enumerate(table):
            if w is EMPTY:
                continue
            a, (r, tag) = slot // sc.B, w
            k = self.decode.get((tag, a, r))
            if k is None:
                self.errors.append(f"slot {slot} holds {w}, which is no key's form under its tag")
                return
            stored.append((k, tag))
        keys = [k for k, _ in stored]
        if len(set(keys)) != len(keys):
            self.errors.append(f"a key is stored twice: {sorted(keys)}")
            return
        expected = set(sc.prefill.values()) | set(sc.ops)
        n_full = results.count(FULL)
        if not set(keys) <= expected or len(keys) != len(expected) - n_full:
            self.errors.append(f"key set {sorted(keys)} is not the {len(expected)} put and pre-filled keys "
                               f"minus one per FULL ({n_full}): a key was lost or made up")
            return
        for k, tag in stored:
            for jj in range(tag):  # every earlier bucket of the key is full
                a = self._bucket_of(k, jj)
                if any(w is EMPTY for w in table[a * sc.B:(a + 1) * sc.B]):
                    self.errors.append(f"key {k} stored under hash {tag} but its bucket for hash {jj} "
                                       f"is not full: the lookup would stop there")
                    return
        for k in expected:
            if self._lookup(table, k) != (1 if k in keys else 0):
                self.errors.append(f"lookup of {k} disagrees with the table")
                return
        if sc.expect_no_full and n_full:
            self.errors.append(f"FULL with room in the table: {results}")


def check(sc: CuckooScenario, limit: int = 3_000_000):
    c = CuckooChecker(sc)
    ok = c.run(limit)
    return ok, c.errors, c.states, c.terminal
