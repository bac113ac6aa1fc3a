"""CPU model of the k-core push step's workgroup-local cascade queue.

The device code (kpeel_push in the k-core source) lets a workgroup delete,
within the same step, low-degree vertices that its own decrements activate:
each wavefront's leader reserves queue slots and arc budget with LDS atomics,
every lane that wanted a slot writes it (its vertex, or -1 when over the arc
budget), and the workgroup drains the queue in rounds [head, tail) between
barriers until no round adds more.  Vertices that get no slot (queue full or
over budget) go to the next step's list instead.

This model runs the same protocol with the wavefronts of one workgroup
interleaved in random order at every point where the hardware may reorder
them (between atomics; barriers are the only synchronisation), for tiny
queues (2, 3 entries) and budgets, and checks the invariants the result
depends on: every slot a drain round reads below min(tail, capacity) has
been written; every activated vertex is deleted exactly once (by the local
drain or by a later step); and the level's deletions equal a sequential
peel's.  It models the protocol, not the memory system: loads and atomics on
one address are taken as sequentially consistent (what the LDS atomics and
the device-scope degree atomics provide for a single address)."""
from __future__ import annotations

import random

import numpy as np
import pytest

from paper_1812_04070_amd import gen


def _sequential_level(off, idx, deg, alive, k):
    """Vertices deleted at level k by repeated deletion of degree <= k."""
    deg = deg.copy()
    alive = alive.copy()
    out = set()
    changed = True
    while changed:
        changed = False
        for v in np.nonzero(alive)[0]:
            if deg[v] <= k:
                alive[v] = False
                out.add(int(v))
                changed = True
                for u in idx[off[v]:off[v + 1]]:
                    if alive[u]:
                        deg[u] -= 1
    return out


class Workgroup:
    """One workgroup's push step with its local queue (the model)."""

    def __init__(self, q_cap, arc_budget, local_deg, rng):
        self.q_cap, self.arc_budget, self.local_deg, self.rng = q_cap, arc_budget, local_deg, rng

    def step(self, frontier, off, idx, deg, state, k, waves=4, lanes=4):
        """Push the vertices of `frontier`; returns (deleted locally, next list)."""
        lq = [None] * self.q_cap          # None: never written
        tail = [0]
        arcs = [0]
        next_list = []
        local_done = []

        def activate(batch):
            # one wavefront's activations: the leader's two atomics (slots,
            # then arc budget), then each wanting lane's slot write.  The two
            # atomics are modelled back to back; another wavefront's between
            # them only changes which lanes are over budget, and each
            # reserved slot is written by its owner either way.
            want = [(u, du) for (u, du) in batch if du < self.local_deg]
            local = {}
            if want:
                base = tail[0]
                tail[0] += len(want)
                incl, s = [], 0
                for _, du in want:
                    s += du
                    incl.append(s)
                abase = arcs[0]
                arcs[0] += s
                for r, (u, du) in enumerate(want):
                    pos = base + r
                    if pos < self.q_cap:
                        ok = abase + incl[r] <= self.arc_budget
                        lq[pos] = u if ok else -1
                        local[u] = ok
            for u, _ in batch:
                if local.get(u, False):
                    state[u] = "local"
                else:
                    state[u] = "next"
                    next_list.append(u)

        def push_vertices(vs):
            # split over the wavefronts; every arc's decrement is one atomic,
            # the wavefronts interleave between them
            jobs = [[] for _ in range(waves)]
            for i, v in enumerate(vs):
                jobs[i % waves].append(v)
            work = []
            for w, vv in enumerate(jobs):
                arcs_w = [(v, u) for v in vv for u in idx[off[v]:off[v + 1]]]
                batches = [arcs_w[i:i + lanes] for i in range(0, len(arcs_w), lanes)]
                work.append(batches)
            while any(work):
                w = self.rng.choice([i for i, b in enumerate(work) if b])
                batch = work[w].pop(0)
                acts = []
                for v, u in batch:
                    if deg[u] > k:                 # the stale-read pre-check
                        old = deg[u]
                        deg[u] -= 1                # atomic decrement
                        if old == k + 1:
                            acts.append((u, int(off[u + 1] - off[u])))
                activate(acts)

        push_vertices(frontier)
        head = 0
        while True:                                # drain rounds, barrier-separated
            t = min(tail[0], self.q_cap)
            if head >= t:
                break
            chunk = lq[head:t]
            assert all(x is not None for x in chunk), "drain read an unwritten slot"
            vs = [x for x in chunk if x >= 0]
            local_done += vs
            push_vertices(vs)
            head = t
        return local_done, next_list


@pytest.mark.parametrize("q_cap,arc_budget", [(2, 1000), (2, 3), (3, 5), (8, 6), (64, 10_000)])
@pytest.mark.parametrize("seed", range(6))
def test_local_queue_protocol(q_cap, arc_budget, seed):
    rng = random.Random(seed * 101 + q_cap)
    g = [gen.random_graph(40, 0.12, seed=seed), gen.rmat(7, seed=seed + 1),
         gen.grid(7, 0.2, seed=seed + 2)][seed % 3]
    off, idx = g.offsets, g.indices
    n = g.n
    deg = np.diff(off).astype(np.int64)
    alive = np.ones(n, dtype=bool)
    core = np.full(n, -1)
    for k in range(0, int(deg.max()) + 2):
        expect = _sequential_level(off, idx, deg, alive, k)
        wg = Workgroup(q_cap, arc_budget, local_deg=4, rng=rng)
        state = {}
        frontier = [int(v) for v in np.nonzero(alive & (deg <= k))[0]]
        for v in frontier:
            state[v] = "scan"
        deleted = []
        while frontier:
            loc, nxt = wg.step(frontier, off, idx, deg, state, k)
            deleted += frontier + loc
            # each vertex is deleted once: no repeats within or across steps
            assert len(set(loc)) == len(loc) and len(set(nxt)) == len(nxt)
            assert not set(loc) & set(nxt)
            frontier = nxt
        assert len(deleted) == len(set(deleted))
        assert set(deleted) == expect, (k, sorted(set(deleted) ^ expect))
        for v in deleted:
            alive[v] = False
            core[v] = k
        if not alive.any():
            break
    assert (core >= 0).all()
