"""A step-level model of the serving loop's resident protocol (the host
dispatcher, the persistent launch's leader block and its worker blocks),
run under many seeded random interleavings on the CPU (an actor, once
chosen, runs for a random burst of steps).

Every shared-memory access of the protocol is one atomic step of an actor
(a Python generator); a scheduler picks the next actor at random.  The model
follows the device code's order of accesses: the leader restarts the ticket
count at the last published chunk and then opens the launch (run_epoch),
mirrors descriptors, publishes their chunk range, and ends the launch
(stop_epoch) when idle or asked to; a worker waits for the launch to open,
takes a ticket (atomic add), waits until that chunk is published or the
launch ends (re-reading the published count after seeing the end), finds
the chunk's descriptor among the last RING mirrored, processes it and counts
it on its slot; the block that reaches the slot's running total reports the
request.  The host publishes descriptors into free slots with chunk sizes
taken from the work in flight and relaunches the loop when requests are in
flight and the leader of the current launch has written that it ended; a
launch starts once the previous one's blocks have all finished (one
stream).

Checked: every published chunk is processed exactly once, by one block;
every request completes, with its done word set only after all its chunks
were processed; no worker misses its descriptor; every launch ends.  The
model is sequentially consistent: it checks the protocol's logic, not the
fences that make it hold on the device.  Two planted mistakes (a leader
that does not restart the ticket count, a worker that gives its ticket up
without re-reading the published count) must each be caught.
"""
from __future__ import annotations

import random
import sys

import pytest

RING = 4          # ring slots (small, so the ring wraps often)
COPY_MAX = 2      # descriptors the leader copies per iteration
IDLE_ITERS = 6    # leader iterations without progress before the launch ends
BURSTS = (1, 1, 1, 2, 3, 8, 40)  # steps an actor runs once chosen


class Shared:
    def __init__(self):
        # host ring
        self.published = 0
        self.stop = 0
        self.done = [0] * RING
        self.desc_host = [None] * RING
        # device state
        self.pub_chunks = 0
        self.mirrored = 0
        self.stop_epoch = 0
        self.run_epoch = 0
        self.next_chunk = 0
        self.slot_done = [0] * RING
        self.desc_dev = [None] * RING
        # observations
        self.processed = {}      # chunk id -> count
        self.fault = False
        self.ended = 0           # epoch of the last launch whose leader ended it


def leader(S, epoch, bug):
    if not bug.get("no_ticket_reset"):
        pc = S.pub_chunks
        yield
        S.next_chunk = pc
        yield
    S.run_epoch = epoch
    yield
    m = S.mirrored
    last_claim = S.next_chunk
    quiet = 0
    while True:
        pub = S.published
        stop = S.stop
        yield
        n_copy = min(max(pub - m, 0), COPY_MAX)
        end = None
        for q in range(m, m + n_copy):
            d = S.desc_host[q % RING]
            yield
            S.desc_dev[q % RING] = dict(d)
            end = d["chunk_base"] + d["chunks"]
            yield
        progress = False
        if n_copy:
            m += n_copy
            S.mirrored = m
            yield
            S.pub_chunks = end
            yield
            progress = True
        claim = S.next_chunk
        yield
        if claim != last_claim:
            last_claim = claim
            progress = True
        quiet = 0 if progress else quiet + 1
        if stop or quiet > IDLE_ITERS:
            S.stop_epoch = epoch
            yield
            S.ended = epoch
            yield
            return


def worker(S, epoch, bug):
    while S.run_epoch != epoch:
        yield
    seq = 0
    while True:
        ticket = S.next_chunk  # fetch-and-add: one atomic step
        S.next_chunk = ticket + 1
        yield
        got = False
        while True:
            pc = S.pub_chunks
            yield
            if ticket < pc:
                got = True
                break
            se = S.stop_epoch
            yield
            if se == epoch:
                if not bug.get("no_recheck"):
                    pc = S.pub_chunks
                    yield
                    got = ticket < pc
                break
        if not got:
            return
        m = S.mirrored
        yield
        if m > RING and seq < m - RING:
            seq = m - RING
        d = None
        while seq < m:
            c = S.desc_dev[seq % RING]
            yield
            if c is not None and c["seq"] == seq and c["chunk_base"] <= ticket < c["chunk_base"] + c["chunks"]:
                d = c
                break
            seq += 1
        if d is None:
            S.fault = True
            return
        S.processed[ticket] = S.processed.get(ticket, 0) + 1
        yield
        slot = d["seq"] % RING
        before = S.slot_done[slot]  # fetch-and-add: one atomic step
        S.slot_done[slot] = before + 1
        yield
        if before + 1 == d["slot_target"]:
            # every chunk of the request was counted after it was processed
            first = d["chunk_base"]
            assert all(S.processed.get(c, 0) == 1 for c in range(first, first + d["chunks"]))
            S.done[slot] = d["seq"] + 1
            yield


def run_model(seed, n_req=40, workers=3, bug=None):
    """One random interleaving; returns the shared state and the requests."""
    bug = bug or {}
    rng = random.Random(seed)
    S = Shared()
    sizes = [rng.randint(1, 9) for _ in range(n_req)]
    next_req = 0
    inflight = {}      # seq -> (slot, ops)
    slot_busy = [False] * RING
    slot_total = [0] * RING
    next_seq = 0
    next_chunk = 0
    inflight_ops = 0
    completed = []
    launches = []      # lists of generators (None once finished), one list per launch, in stream order
    running = 0        # launches before this one have finished; it runs once launched
    epoch = 0
    steps = 0
    while True:
        steps += 1
        assert steps < 200000, "no progress"
        # launches run one after another on the stream
        while running < len(launches) and all(g is None for g in launches[running]):
            running += 1
        live = [g for g in launches[running] if g is not None] if running < len(launches) else []
        # the host is one more actor
        actors = ["host"] + list(range(len(live)))
        a = rng.choice(actors)
        if a == "host":
            # completions
            for q in list(inflight):
                slot, ops = inflight[q]
                if S.done[slot] == q + 1:
                    del inflight[q]
                    slot_busy[slot] = False
                    inflight_ops -= ops
                    completed.append(q)
            # admit a random number of requests into free slots (arrivals come in bursts)
            take = []
            for _ in range(rng.randint(0, 2)):
                if next_req < n_req and not slot_busy[next_seq % RING]:
                    slot = next_seq % RING
                    slot_busy[slot] = True
                    take.append((next_seq, slot, sizes[next_req]))
                    next_seq += 1
                    next_req += 1
            inflight_ops += sum(t[2] for t in take)
            per_worker = -(-inflight_ops // workers) if take else 0
            lg = 0
            while lg < 2 and (1 << lg) < per_worker:
                lg += 1
            for q, slot, ops in take:
                chunks = -(-ops // (1 << lg))
                slot_total[slot] += chunks
                S.desc_host[slot] = dict(seq=q, chunk_base=next_chunk, chunks=chunks, slot_target=slot_total[slot])
                next_chunk += chunks
                inflight[q] = (slot, ops)
            if take:
                S.published = next_seq
            # relaunch when requests are in flight and the current launch's
            # leader has ended it (its last blocks may still run: the new
            # launch queues behind them)
            if inflight and (epoch == 0 or S.ended == epoch):
                epoch += 1
                launches.append([leader(S, epoch, bug)] + [worker(S, epoch, bug) for _ in range(workers)])
            if next_req == n_req and not inflight and not live and running == len(launches):
                break
            continue
        g = live[a]
        # run the chosen block for a burst of steps: long bursts let one
        # actor get far ahead of another, which is where races show
        for _ in range(rng.choice(BURSTS)):
            try:
                next(g)
            except StopIteration:
                cur = launches[running]
                cur[cur.index(g)] = None
                break
        if S.fault:
            break
    return S, next_chunk, completed, len(launches)


@pytest.mark.parametrize("seed", range(300))
def test_resident_protocol_exactly_once(seed):
    S, n_chunks, completed, n_launch = run_model(seed, workers=1 + seed % 4)
    assert not S.fault, "a worker did not find its descriptor"
    assert sorted(completed) == list(range(40)), "every request completes"
    assert sorted(S.processed) == list(range(n_chunks)), "every published chunk is processed"
    assert all(v == 1 for v in S.processed.values()), "no chunk is processed twice"
    assert n_launch >= 1


@pytest.mark.parametrize("seed", range(40))
def test_resident_protocol_larger_ring(seed, monkeypatch):
    """The same checks with a 16-slot ring, copies of up to 8 descriptors per
    leader pass, 200 requests and up to 8 workers."""
    mod = sys.modules[__name__]
    monkeypatch.setattr(mod, "RING", 16)
    monkeypatch.setattr(mod, "COPY_MAX", 8)
    assert Shared().done == [0] * 16
    S, n_chunks, completed, _ = run_model(seed, n_req=200, workers=1 + seed % 8)
    assert not S.fault
    assert sorted(completed) == list(range(200))
    assert sorted(S.processed) == list(range(n_chunks))
    assert all(v == 1 for v in S.processed.values())


def _fails(bug, seeds=range(200)):
    for seed in seeds:
        try:
            S, n_chunks, completed, _ = run_model(seed, workers=1 + seed % 4, bug=bug)
        except AssertionError:
            return True
        if S.fault or sorted(completed) != list(range(40)) or sorted(S.processed) != list(range(n_chunks)) \
                or any(v != 1 for v in S.processed.values()):
            return True
    return False


def test_model_catches_a_leader_that_keeps_stale_tickets():
    """Without the restart, the tickets a launch gave up are never handed out
    again, so their chunks are never processed (the requests hang)."""
    assert _fails({"no_ticket_reset": True})


def test_model_catches_a_worker_that_gives_up_a_published_ticket():
    """A worker that sees the launch end and leaves without re-reading the
    published count can drop a chunk published just before the end."""
    assert _fails({"no_recheck": True})
