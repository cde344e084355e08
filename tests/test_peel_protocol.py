"""Host model of the grid PeelOne's claim protocol (Alg. 4 with the
assertion decrement and the dynamic frontier, Section III), run under
randomised interleavings.

The GPU kernel overlaps a level's scan with the expansion of what the scan
found: a scanner claims a vertex it reads at value k with a compare-and-swap,
and a decrement claims the vertex its fetch took from k + 1 to k, or found at
exactly k, also with a compare-and-swap.  Batches expanded inside a workgroup
decrement every neighbour without reading its value first; the shared
edge-balanced rounds read it and skip neighbours valued k or less.  Once the
scan phase has ended (a grid barrier), the kernel claims with a plain store:
only the fetch that returns k + 1 claims.  This model replays those rules
with the scan reads, the local expansions and the rounds' entries taken in
random order, and checks that no vertex is ever claimed twice, that each is
claimed at its coreness, and that no vertex receives more decrements than its
degree.  It models the protocol's logic, not the memory system: each read
sees the latest value, except that the rounds' filter may read a value from
the start of the round (a stale read).
"""
import random

import numpy as np
import pytest

import graphgen as gg
import oracle


class DoubleClaim(AssertionError):
    pass


def _peel_model(off, adj, seed, local_share=0.6, round_claims_at_k=False):
    """Coreness by the kernel's level protocol under one random interleaving
    (each read, fetch-and-subtract and compare-and-swap is one event).
    round_claims_at_k: a deliberately wrong variant whose rounds also claim on
    a fetch that returns k (must be caught)."""
    rng = random.Random(seed)
    n = off.shape[0] - 1
    deg = np.diff(off)
    core = deg.astype(np.int64).copy()
    out = np.full(n, -1, dtype=np.int64)
    out[deg == 0] = 0
    decs = np.zeros(n, dtype=np.int64)
    blocks = 4
    state = {"k": 0, "scanning": True}
    queues = [[] for _ in range(blocks)]
    glob = []

    def nbrs(v):
        return [int(u) for u in adj[off[v]:off[v + 1]]]

    def decrement(u):
        old = int(core[u])
        core[u] -= 1
        decs[u] += 1
        return old

    def claim_cas(v):
        if out[v] == -1:
            out[v] = state["k"]
            return True
        return False

    def claim_plain(v):
        if out[v] != -1:
            raise DoubleClaim(f"vertex {v} claimed at level {out[v]} and again at {state['k']}")
        out[v] = state["k"]

    def assert_into_frontier(v):
        b = rng.randrange(blocks)
        (queues[b] if rng.random() < local_share else glob).append(v)

    def expand_local(b):
        v = queues[b].pop(rng.randrange(len(queues[b])))
        k = state["k"]
        for u in nbrs(v):
            old = decrement(u)  # no filter read in a local batch
            if state["scanning"]:
                if old in (k + 1, k) and claim_cas(u):
                    assert_into_frontier(u)
            elif old == k + 1 or (round_claims_at_k and old == k):
                claim_plain(u)
                assert_into_frontier(u)

    def busy():
        return [i for i in range(blocks) if queues[i]]

    survivors = [v for v in range(n) if deg[v] > 0]
    k = int(min(core[v] for v in survivors)) if survivors else 0
    while survivors:
        state["k"], state["scanning"] = k, True
        # scan phase: every survivor is read once, interleaved with the
        # workgroups' expansion of what they have found so far
        pending = list(survivors)
        rng.shuffle(pending)
        while pending or busy():
            if pending and (not busy() or rng.random() < 0.5):
                v = pending.pop()
                if core[v] == k and claim_cas(v):
                    assert_into_frontier(v)
            else:
                expand_local(rng.choice(busy()))
        # grid barrier: every vertex valued k or less is claimed by now
        assert all(out[v] != -1 for v in survivors if core[v] <= k)
        state["scanning"] = False
        # rounds over the shared list; the filter may read the round's start value
        while glob:
            entries = glob[:]
            glob.clear()
            start = core.copy()
            work = [(v, u) for v in entries for u in nbrs(v)]
            rng.shuffle(work)
            for v, u in work:
                seen = start[u] if rng.random() < 0.5 else core[u]
                if seen > k:
                    old = decrement(u)
                    if old == k + 1 or (round_claims_at_k and old == k):
                        claim_plain(u)
                        assert_into_frontier(u)
            while busy():
                expand_local(rng.choice(busy()))
        survivors = [v for v in survivors if out[v] == -1]
        assert all(core[v] > k for v in survivors)
        k += 1
    assert (decs <= deg).all()
    return out


GRAPHS = [lambda: gg.er_gnp(300, 6.0, 11), lambda: gg.rmat(9, 8, 4),
          lambda: gg.disjoint_union(gg.complete(12), gg.cycle(20), gg.star(30)),
          lambda: gg.scaled_rmat_block(9, 3, 40, 0.7, 5)]


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("make", GRAPHS)
def test_claim_protocol_matches_bz(make, seed):
    g = make()
    off = g.offsets.numpy().astype(np.int64)
    adj = g.cols.numpy()
    want = oracle.bz_coreness(g.offsets, g.cols)
    for local_share in (0.0, 0.6, 1.0):
        got = _peel_model(off, adj, seed * 7 + int(local_share * 10), local_share=local_share)
        assert np.array_equal(got, want), (g.name, seed, local_share)


def test_claim_protocol_catches_a_claim_at_k_in_rounds():
    """The model is sharp: rounds that also claimed on a fetch returning k (as
    the scan phase may, guarded by its compare-and-swap) claim some vertex
    twice on these interleavings."""
    g = gg.scaled_rmat_block(9, 3, 40, 0.7, 5)
    off = g.offsets.numpy().astype(np.int64)
    adj = g.cols.numpy()
    with pytest.raises(DoubleClaim):
        for seed in range(20):
            _peel_model(off, adj, seed, local_share=0.3, round_claims_at_k=True)

