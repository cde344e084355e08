"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests touches a GPU.  The oracle is only trusted because it
passes them: worked-example values printed in the paper (G1, Fig. 1 / Fig. 6 /
the PeelOne narrative), brute force on every labelled graph with up to six
vertices and on random graphs up to fourteen, closed forms of textbook
families, and cross-checks between independent routines (bucket peel vs
synchronous h-index iteration vs serial PeelOne vs serial HistoCore).
"""
import itertools
import random

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle


def _edges_of(g):
    s, d = g.edge_pairs()
    return [(int(a), int(b)) for a, b in zip(s.tolist(), d.tolist()) if a < b]


# ---------------------------------------------------------------- worked example G1

def test_g1_coreness_all_routines(golden_g1):
    g = gg.g1()
    want = [int(x) for x in golden_g1["coreness"]]
    edges = [tuple(int(t) for t in e.split("-")) for e in golden_g1["edges"]]
    assert sorted(edges) == sorted(_edges_of(g))
    assert oracle.bz_coreness(g.offsets, g.cols).tolist() == want
    assert oracle.brute_coreness(6, edges) == want
    assert oracle.peelone_trace(g.offsets, g.cols)["core"] == want
    assert oracle.histocore_trace(g.offsets, g.cols)["core"] == want
    x, _, _ = oracle.hindex_jacobi(g.offsets, g.cols)
    assert x.tolist() == want


def test_g1_under_core_vertices(golden_g1):
    """Removing the vertices of coreness <= 2 found by the scans of iterations 1
    and 2 of the general parallel peel (v0, v1, then v2, v4) leaves v3 and v5
    with residual degree 1 < coreness 2: the under-core set (Section III-A)."""
    g = gg.g1()
    core = oracle.bz_coreness(g.offsets, g.cols)
    removed = {0, 1, 2, 4}
    under = []
    for v in range(6):
        if v in removed:
            continue
        res_deg = sum(1 for u in g.cols[g.offsets[v]:g.offsets[v + 1]].tolist() if u not in removed)
        if res_deg < core[v]:
            under.append(v)
    assert under == [int(x) for x in golden_g1["under_core"]]


def test_g1_peelone_trace(golden_g1):
    t = oracle.peelone_trace(gg.g1().offsets, gg.g1().cols)
    lv = {L["k"]: L for L in t["levels"]}
    assert lv[2]["scan"] == [int(x) for x in golden_g1["peelone_k2_scan"]]
    assert sorted(lv[2]["dynamic"]) == [int(x) for x in golden_g1["peelone_k2_dynamic"]]
    assert lv[1]["scan"] == [0, 1] and lv[1]["dynamic"] == []
    # v5: 5 -> 4 -> 3 during level 1, 3 -> 2 by the assertion decrement at level 2
    assert t["trajectory"][5] == [5, 4, 3, 2]
    assert t["trajectory"][3] == [3, 2]
    assert len(t["levels"]) == 2  # levels = k_max (Table V: l1 equals k_max)


def test_g1_histocore_trace(golden_g1):
    g = gg.g1()
    t = oracle.histocore_trace(g.offsets, g.cols)
    want = {int(a): int(b) for a, b in (p.split(":") for p in golden_g1["v5_histogram"])}
    h5 = t["init_histo"][5]
    assert {i: h5[i] for i in range(1, 6) if h5[i]} == want
    assert t["frontiers"] == [[3, 5]]
    assert t["iterations"] == 1
    assert t["cnt_ok"]
    x1, per_round, last = oracle.hindex_jacobi(g.offsets, g.cols, max_rounds=1)
    a, b = (int(v) for v in golden_g1["v5_round1_change"])
    assert g.degrees()[5].item() == a and x1[5] == b == int(golden_g1["v5_hindex_round1"][0])
    # v0, v1, v2, v4 never change (Section II-C: they need no re-estimation)
    _, per_round, last = oracle.hindex_jacobi(g.offsets, g.cols)
    assert [v for v in range(6) if last[v] == 0] == [0, 1, 2, 4]
    assert per_round == [2]


# ---------------------------------------------------------------- brute force

def _all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        yield [p for i, p in enumerate(pairs) if mask >> i & 1]


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 6])
def test_bz_equals_brute_force_exhaustive(n):
    for edges in _all_graphs(n):
        g = gg.from_edge_list(n, edges)
        got = oracle.bz_coreness(g.offsets, g.cols).tolist()
        assert got == oracle.brute_coreness(n, edges), (n, edges)


def test_bz_equals_brute_force_random():
    rng = random.Random(14)
    for trial in range(10000):
        n = rng.randint(1, 14)
        p = rng.random()
        edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
        g = gg.from_edge_list(n, edges)
        assert oracle.bz_coreness(g.offsets, g.cols).tolist() == oracle.brute_coreness(n, edges)


# ---------------------------------------------------------------- closed forms

def _core(g):
    return oracle.bz_coreness(g.offsets, g.cols)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 40])
def test_complete_graph(n):
    assert (_core(gg.complete(n)) == n - 1).all()


@pytest.mark.parametrize("n", [3, 4, 11, 1000])
def test_cycle(n):
    assert (_core(gg.cycle(n)) == 2).all()


def test_path_star_tree():
    assert (_core(gg.path(5000)) == 1).all()
    assert (_core(gg.star(100000)) == 1).all()
    rng = random.Random(3)
    n = 3000
    edges = [(v, rng.randrange(v)) for v in range(1, n)]  # random recursive tree
    assert (_core(gg.from_edge_list(n, edges)) == 1).all()


def test_isolated_and_empty():
    assert _core(gg.empty_graph(0)).tolist() == []
    assert (_core(gg.empty_graph(17)) == 0).all()
    g = gg.from_edge_list(5, [(1, 3)])
    assert _core(g).tolist() == [0, 1, 0, 1, 0]


@pytest.mark.parametrize("a,b", [(1, 1), (1, 9), (3, 5), (7, 7), (12, 30)])
def test_complete_bipartite(a, b):
    assert (_core(gg.complete_bipartite(a, b)) == min(a, b)).all()


@pytest.mark.parametrize("d", [0, 1, 2, 5, 10])
def test_hypercube_is_d(d):
    assert (_core(gg.hypercube(d)) == d).all()


def test_circulant_regular():
    g = gg.circulant(101, [1, 2, 5, 13])  # connected 8-regular
    assert (_core(g) == 8).all()


def test_disjoint_union_is_per_component():
    parts = [gg.complete(9), gg.cycle(20), gg.star(7), gg.hypercube(4), gg.empty_graph(3)]
    g = gg.disjoint_union(*parts)
    want = np.concatenate([_core(p) for p in parts])
    assert (_core(g) == want).all()
    assert want[:9].tolist() == [8] * 9


# ---------------------------------------------------------------- cross-checks

def _random_graphs():
    out = [gg.er_gnp(300, 6.0, s) for s in range(4)]
    out += [gg.rmat(10, 8, s) for s in range(4)]
    out.append(gg.scaled_rmat_block(11, 5, 60, 0.5, 9))
    out.append(gg.disjoint_union(gg.path(200), gg.complete(30), gg.star(50)))
    return out


@pytest.mark.parametrize("g", _random_graphs(), ids=lambda g: g.name)
def test_independent_routines_agree(g):
    """Bucket peel, h-index fixed point (Index2core reaches coreness), serial
    PeelOne and serial HistoCore all give the same vector."""
    core = _core(g)
    x, per_round, last = oracle.hindex_jacobi(g.offsets, g.cols)
    assert (x == core).all()
    po = oracle.peelone_trace(g.offsets, g.cols)
    assert po["core"] == core.tolist()
    hc = oracle.histocore_trace(g.offsets, g.cols)
    assert hc["core"] == core.tolist()
    # Theorem 2: HistoCore's frontier of iteration t is exactly the set of
    # vertices whose h-index changes in synchronous round t.
    assert hc["iterations"] == len(per_round)
    for t, fr in enumerate(hc["frontiers"], start=1):
        assert len(fr) == per_round[t - 1]
    for v in range(g.n):
        rounds_v = [t for t, fr in enumerate(hc["frontiers"], start=1) if v in set(fr)]
        assert (rounds_v[-1] if rounds_v else 0) == last[v]
    assert hc["cnt_ok"]
    # PeelOne: level k peels exactly {v : core(v) = k}, each vertex once, and
    # the level count is k_max (Table V: l1 equals k_max).
    seen = []
    for L in po["levels"]:
        got = sorted(L["scan"] + L["dynamic"])
        assert got == sorted(np.nonzero(core == L["k"])[0].tolist())
        seen += got
    assert sorted(seen) == sorted(np.nonzero(core > 0)[0].tolist())
    assert len(po["levels"]) == int(core.max(initial=0))
    # Corollary 1: no value ever drops below the level at which it is peeled.
    for v in range(g.n):
        assert min(po["trajectory"][v]) >= core[v]


def test_hindex_rounds_monotone():
    g = gg.rmat(11, 8, 1)
    prev = g.degrees().numpy()
    _, per_round, _ = oracle.hindex_jacobi(g.offsets, g.cols)
    for t in range(1, len(per_round) + 1):
        x, _, _ = oracle.hindex_jacobi(g.offsets, g.cols, max_rounds=t)
        assert (x <= prev).all() and int((x != prev).sum()) == per_round[t - 1]
        prev = x


def test_invariants_on_er10k():
    g = gg.er_10k()
    core = _core(g)
    deg = g.degrees().numpy()
    off = g.offsets.numpy().astype(np.int64)
    cols = g.cols.numpy()
    assert (core <= deg).all()
    src = np.repeat(np.arange(g.n), deg)
    # min degree >= k inside {core >= k}
    for k in range(1, int(core.max()) + 1):
        inside = core >= k
        d_in = np.bincount(src[inside[src] & inside[cols]], minlength=g.n)
        assert (d_in[inside] >= k).all()
    # fixed point of the h-index operator
    for v in range(g.n):
        vals = np.sort(core[cols[off[v]:off[v + 1]]])[::-1]
        h = 0
        while h < len(vals) and vals[h] >= h + 1:
            h += 1
        assert h == core[v]
    assert int((deg == 0).sum()) == int((core == 0).sum())


def test_planted_mistake_is_caught():
    """A peel that forgets the 'only neighbours ranked above' guard (a plausible
    slip) disagrees with brute force on some six-vertex graph."""
    def bad_peel(n, edges):
        nbr = [set() for _ in range(n)]
        for u, v in edges:
            nbr[u].add(v); nbr[v].add(u)
        deg = [len(s) for s in nbr]
        alive = set(range(n))
        core = [0] * n
        while alive:
            v = min(alive, key=lambda x: (deg[x], x))
            core[v] = deg[v]
            alive.discard(v)
            for u in nbr[v]:
                if u in alive:
                    deg[u] -= 1  # should not drop below deg[v]
        return core
    caught = any(bad_peel(6, e) != oracle.brute_coreness(6, e) for e in _all_graphs(6))
    assert caught


# ---------------------------------------------------------------- core maintenance
# The iteration from upper bounds (hindex_jacobi_from) is pinned to the plain
# iteration from the degrees, to BZ and brute force on the changed graph, and
# to the facts that make it a maintenance method: deleting edges never raises
# a coreness, one insertion raises any coreness by at most one, and a start
# below the coreness is not repaired (values never rise).

MAINT_GRAPHS = [lambda: gg.rmat(10, 8, 3), lambda: gg.er_gnp(600, 6.0, 4), lambda: gg.g1(),
                lambda: gg.disjoint_union(gg.complete(12), gg.cycle(9), gg.star(20), gg.empty_graph(3))]


@pytest.mark.parametrize("gi", range(len(MAINT_GRAPHS)))
def test_jacobi_from_degrees_is_the_plain_iteration(gi):
    g = MAINT_GRAPHS[gi]()
    x, pr, last = oracle.hindex_jacobi(g.offsets, g.cols)
    deg = g.degrees().numpy().astype(np.int32)
    y, pr2, last2 = oracle.hindex_jacobi_from(g.offsets, g.cols, deg)
    assert np.array_equal(x, y) and pr == pr2 and np.array_equal(last, last2)
    # any start at or above the degree is capped to it
    z, pr3, _ = oracle.hindex_jacobi_from(g.offsets, g.cols, deg, add=1000)
    assert np.array_equal(x, z) and pr == pr3


@pytest.mark.parametrize("gi", range(len(MAINT_GRAPHS)))
@pytest.mark.parametrize("add", [0, 1, 7])
def test_jacobi_from_upper_bounds_reaches_coreness(gi, add):
    g = MAINT_GRAPHS[gi]()
    core = oracle.bz_coreness(g.offsets, g.cols)
    x, pr, _ = oracle.hindex_jacobi_from(g.offsets, g.cols, core, add=add)
    assert np.array_equal(x, core)
    if add == 0:
        assert pr == []  # the coreness is a fixed point: nothing changes


@pytest.mark.parametrize("seed", range(6))
def test_maintenance_after_deletions_and_insertions(seed):
    g = gg.rmat(11, 8, 40 + seed) if seed % 2 else gg.er_gnp(1500, 8.0, 40 + seed)
    old = oracle.bz_coreness(g.offsets, g.cols)
    # deletions only: the old coreness bounds the new one
    h, ins = gg.edit_edges(g, 0.03, 0, seed)
    assert ins == 0 and h.m < g.m
    new = oracle.bz_coreness(h.offsets, h.cols)
    assert (new <= old).all()
    x, pr, _ = oracle.hindex_jacobi_from(h.offsets, h.cols, old)
    assert np.array_equal(x, new)
    cold = oracle.hindex_jacobi(h.offsets, h.cols)[1]
    assert len(pr) <= len(cold) and sum(pr) <= sum(cold)
    # deletions and b insertions: old + b bounds the new coreness
    h2, b = gg.edit_edges(g, 0.01, 25, seed)
    assert b > 0
    new2 = oracle.bz_coreness(h2.offsets, h2.cols)
    assert (new2 <= old + b).all()
    x2, _, _ = oracle.hindex_jacobi_from(h2.offsets, h2.cols, old, add=b)
    assert np.array_equal(x2, new2)


def test_one_insertion_raises_coreness_by_at_most_one():
    g = gg.er_gnp(300, 5.0, 9)
    core = oracle.bz_coreness(g.offsets, g.cols)
    for trial in range(20):
        h, ins = gg.edit_edges(g, 0.0, 1, 100 + trial)
        new = oracle.bz_coreness(h.offsets, h.cols)
        assert ((new - core) >= 0).all() and ((new - core) <= 1).all()
        x, _, _ = oracle.hindex_jacobi_from(h.offsets, h.cols, core, add=ins)
        assert np.array_equal(x, new)


@pytest.mark.parametrize("n", [5, 6, 7])
def test_maintenance_brute_force_tiny(n):
    rng = random.Random(n)
    pairs = list(itertools.combinations(range(n), 2))
    for _ in range(25):
        edges = [p for p in pairs if rng.random() < 0.5]
        g = gg.from_edge_list(n, edges)
        want = oracle.brute_coreness(n, edges)
        # random upper bounds: coreness plus a random non-negative slack
        start = np.array([c + rng.randrange(0, 4) for c in want], dtype=np.int32)
        x, _, _ = oracle.hindex_jacobi_from(g.offsets, g.cols, start)
        assert x.tolist() == want


def test_start_below_coreness_is_not_repaired():
    g = gg.complete(8)  # coreness 7 everywhere
    x, pr, _ = oracle.hindex_jacobi_from(g.offsets, g.cols, np.full(8, 3, dtype=np.int32))
    assert (x == 3).all() and pr == []


# ---------------------------------------------------------------- PeelOne without the dynamic frontier
# (the variant of Table IV): same coreness, more iterations.  Pins: closed
# forms for paths, cycles, cliques and stars, and G1's narrative (Section
# III-C, Fig. 5: at k = 2 the scan finds v2, v4 and v3, v5 only reach 2 during
# the level, so without the dynamic frontier they need a second iteration).

def test_static_peel_g1(golden_g1):
    g = gg.g1()
    x, it = oracle.peel_static(g.offsets, g.cols)
    assert x.tolist() == [int(c) for c in golden_g1["coreness"]]
    levels = len(set(int(c) for c in golden_g1["coreness"] if int(c) > 0))
    assert golden_g1["peelone_k2_dynamic"]  # vertices that wait for a second iteration
    assert it == levels + 1 == 3


@pytest.mark.parametrize("n", [2, 3, 10, 51, 200])
def test_static_peel_path_closed_form(n):
    g = gg.path(n)
    x, it = oracle.peel_static(g.offsets, g.cols)
    assert (x == 1).all()
    assert it == (n + 1) // 2  # the two ends go each iteration


def test_static_peel_closed_forms():
    for g, iters in ((gg.cycle(40), 1), (gg.complete(30), 1), (gg.star(25), 2), (gg.hypercube(5), 1),
                     (gg.empty_graph(4), 0)):
        x, it = oracle.peel_static(g.offsets, g.cols)
        assert np.array_equal(x, oracle.bz_coreness(g.offsets, g.cols)), g.name
        assert it == iters, g.name


@pytest.mark.parametrize("seed", range(4))
def test_static_peel_matches_bz_and_needs_more_iterations(seed):
    g = gg.rmat(11, 8, 60 + seed) if seed % 2 else gg.er_gnp(2000, 6.0, 60 + seed)
    want = oracle.bz_coreness(g.offsets, g.cols)
    x, it = oracle.peel_static(g.offsets, g.cols)
    assert np.array_equal(x, want)
    assert it >= len(np.unique(want[want > 0]))


# ---------------------------------------------------------------- CntCore and NbrCore (Table VI's baselines)
# Pins: the coreness (BZ); Theorem 2 -- CntCore's frontier in each round is
# exactly the set of vertices whose value the synchronous h-index iteration
# lowers, so its rounds and h-index computations equal hindex_jacobi's rounds
# and changed counts; NbrCore recomputes every active vertex and needs one
# more round to see that nothing changes; G1's narrative (Section II-C: only
# v3 and v5 change, v5 from 5 to 2; nobody changes afterwards).

I2C_GRAPHS = [lambda: gg.g1(), lambda: gg.rmat(11, 8, 91), lambda: gg.er_gnp(1500, 7.0, 92),
              lambda: gg.path(101), lambda: gg.complete(20), lambda: gg.star(50),
              lambda: gg.disjoint_union(gg.complete(9), gg.cycle(12), gg.empty_graph(3), gg.hypercube(5))]


@pytest.mark.parametrize("gi", range(len(I2C_GRAPHS)))
def test_cntcore_nbrcore(gi):
    g = I2C_GRAPHS[gi]()
    want = oracle.bz_coreness(g.offsets, g.cols)
    _, per_round, _ = oracle.hindex_jacobi(g.offsets, g.cols)
    xc, c = oracle.index2core(g.offsets, g.cols, "cntcore")
    xn, nb = oracle.index2core(g.offsets, g.cols, "nbrcore")
    assert np.array_equal(xc, want) and np.array_equal(xn, want)
    assert c["rounds_changed"] == nb["rounds_changed"] == len(per_round)
    assert c["hindex_computed"] == sum(per_round)
    live = int((g.degrees() > 0).sum())
    assert nb["hindex_computed"] == nb["active"] >= live
    assert nb["rounds_run"] == (len(per_round) + 1 if live else 0)
    assert c["edges_hindex"] == c["edges_mark"] == nb["edges_mark"]
    assert c["activations"] == nb["activations"] and c["active"] == nb["active"]
    assert nb["edges_hindex"] == c["edges_cnt"]  # same active sets, read once each


def test_cntcore_g1(golden_g1):
    g = gg.g1()
    _, c = oracle.index2core(g.offsets, g.cols, "cntcore")
    under = [int(v) for v in golden_g1["under_core"]]  # v3, v5: the only vertices that change
    assert c["rounds_changed"] == 1 and c["hindex_computed"] == len(under) == 2
    assert c["active"] == 6 + 6  # round 1: every vertex; round 2: the neighbours of v3 and v5


# ---------------------------------------------------------------- General Parallel Peel (Alg. 3)
# Pins: BZ; closed forms; G1 from Section III-A, which states that GPP needs
# three iterations on G1 (Alg. 3 raises k before the scan of the same
# iteration, so the advance from k = 1 to 2 costs no iteration of its own).

def test_gpp_g1_narrative(golden_g1):
    g = gg.g1()
    x, it, dec = oracle.peel_gpp(g.offsets, g.cols)
    assert x.tolist() == [int(c) for c in golden_g1["coreness"]]
    # 1: k 0 -> 1, v0 and v1 (degree 1) go; 2: nobody at or below 1, k -> 2, v2 and
    # v4 go and v3, v5 fall to degree 1 (Section II-C); 3: v3 and v5 go
    assert it == 3
    # decrements: iteration 1 along v0-v5, v1-v5; iteration 2 along v2-v5, v2-v3, v4-v3,
    # v4-v5; v3 and v5 go together in iteration 3, so their edge costs nothing
    assert dec == 6


def test_gpp_closed_forms():
    # path: both ends go in each iteration, the middle vertex of an odd path
    # alone in the last; K_n and d-regular graphs: k rises by one per iteration
    # from 0 to the degree, all removed in the last; star: leaves, then the
    # centre (degree 0 by then) at the same k; isolated vertices only: one
    # iteration at k = 0
    for g, iters in ((gg.path(51), 26), (gg.complete(12), 11), (gg.cycle(30), 2), (gg.star(40), 2),
                     (gg.empty_graph(3), 1), (gg.hypercube(4), 4)):
        x, it, dec = oracle.peel_gpp(g.offsets, g.cols)
        assert np.array_equal(x, oracle.bz_coreness(g.offsets, g.cols)), g.name
        assert it == iters, g.name
        assert dec <= g.m // 2  # at most one decrement per undirected edge


def test_gpp_isolated_vertices_take_the_first_iteration():
    """Alg. 3 starts at k = 0 with every vertex residual: isolated vertices
    leave in the first iteration with coreness 0, which adds exactly one
    iteration to the graph without them."""
    g = gg.path(11)
    _, it, dec = oracle.peel_gpp(g.offsets, g.cols)
    off = np.concatenate([g.offsets.numpy().astype(np.int64), np.full(4, g.m, dtype=np.int64)])
    x2, it2, dec2 = oracle.peel_gpp(off, g.cols.numpy())
    assert it2 == it + 1 and dec2 == dec
    assert x2[-4:].tolist() == [0, 0, 0, 0]


@pytest.mark.parametrize("seed", range(4))
def test_gpp_matches_bz(seed):
    g = gg.rmat(11, 8, 70 + seed) if seed % 2 else gg.er_gnp(2000, 6.0, 70 + seed)
    want = oracle.bz_coreness(g.offsets, g.cols)
    x, it, _ = oracle.peel_gpp(g.offsets, g.cols)
    assert np.array_equal(x, want)
    _, it_static = oracle.peel_static(g.offsets, g.cols)
    assert it >= it_static  # the same removals, plus a scan for every empty level
