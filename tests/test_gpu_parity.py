"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Coreness is integer and unique, so every comparison is bit-exact.  Schedule
statistics are compared where the paper fixes them: PeelOne runs one level per
distinct coreness value (Table V: l1 equals k_max when no level is empty), and
HistoCore's rounds and per-round frontier sizes equal the synchronous h-index
iteration's (Theorem 2).
"""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_2402_15253_amd as pico
from tests.golden.make_schedules import fingerprint

pytestmark = pytest.mark.gpu

ALGOS = ["peelone", "histocore"]


def _gpu(g):
    return g.to("cuda")


def _run(g, algo, with_stats=False, path=None):
    d = _gpu(g)
    res = pico.coreness(d.offsets, d.cols, algo, with_stats=with_stats, path=path)
    torch.cuda.synchronize()
    if with_stats:
        return res[0].cpu().numpy(), res[1]
    return res.cpu().numpy()


def _check(g, algo, path=None):
    want = oracle.bz_coreness(g.offsets, g.cols)
    got, st = _run(g, algo, with_stats=True, path=path)
    assert got.dtype == np.int32 and got.shape == (g.n,)
    mism = np.nonzero(got != want)[0]
    assert mism.size == 0, f"{g.name} {algo}: {mism.size} mismatches, first {mism[:5]} " \
                           f"got {got[mism[:5]]} want {want[mism[:5]]}"
    return want, st


@pytest.mark.parametrize("algo", ALGOS)
def test_g1(algo, golden_g1):
    assert _run(gg.g1(), algo).tolist() == [int(x) for x in golden_g1["coreness"]]


SMALL_CASES = [
    lambda: gg.complete(2), lambda: gg.complete(40), lambda: gg.cycle(1001),
    lambda: gg.star(100_000), lambda: gg.complete_bipartite(12, 300), lambda: gg.hypercube(10),
    lambda: gg.empty_graph(1), lambda: gg.empty_graph(1000), lambda: gg.from_edge_list(7, [(2, 5)]),
    lambda: gg.disjoint_union(gg.complete(60), gg.cycle(30), gg.star(5000), gg.empty_graph(9),
                              gg.hypercube(6)),
    lambda: gg.circulant(5000, [1, 3, 7, 20, 50]),
]


# values of up to this many vertices fit in one workgroup's LDS on gfx950
WG_FITS = 32768


@pytest.mark.parametrize("path", ["grid", "wg"])
@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("case", range(len(SMALL_CASES)))
def test_closed_forms_and_edge_cases(algo, case, path):
    g = SMALL_CASES[case]()
    print(f"case {g.name} n={g.n} m={g.m} algo={algo} path={path}", flush=True)
    if path == "wg" and g.n > 2 * WG_FITS:
        with pytest.raises(pico.PicoError) as e:
            _run(g, algo, path=path)
        assert e.value.status == pico.PICO_ENOTSUP
        return
    _check(g, algo, path)


@pytest.mark.parametrize("algo", ALGOS)
def test_large_clique_one_workgroup(algo):
    g = gg.complete(2000)  # 4M entries, far above the default bound of the path
    got = _run(g, algo, path="wg")
    assert (got == 1999).all()


@pytest.mark.parametrize("offsets_dtype", [torch.int32, torch.int64])
def test_paths_agree_on_schedule(offsets_dtype, monkeypatch):
    """The one-workgroup and grid paths report the same schedule where it is
    fixed by the graph: PeelOne's levels, peeled vertices and k_max;
    HistoCore's rounds, frontier sizes, edges scanned and histogram moves
    (Theorem 2 fixes the synchronous rounds).  PeelOne's split of each level
    between vertices its scan found and vertices a decrement asserted is not
    fixed on the grid path (a workgroup's local batch may decrement and claim
    a vertex valued k before another workgroup's scan reaches it), so only
    its bounds are checked; the per-level totals are compared element by
    element in the schedule tests.  Scan counts may differ by one: the grid
    path ends with a scan that finds no survivor when the last level's
    survivors were all asserted during its drain.  The grid path's histogram
    rebuild rounds are switched off here (they read every entry and move
    nothing); test_rebuild_rounds_keep_the_schedule covers them."""
    monkeypatch.setenv("PICO_HC_REBUILD_PERMILLE", "2000")
    g = gg.rmat(13, 16, 21).with_offsets(offsets_dtype)
    print(f"case {g.name} n={g.n} m={g.m} {offsets_dtype}", flush=True)
    for algo, keys in (("peelone", ("iterations", "frontier_total", "k_max", "edges_scanned")),
                       ("histocore", ("iterations", "frontier_total", "edges_scanned", "atomics",
                                      "pushes_dynamic"))):
        _, st_wg = _check(g, algo, "wg")
        _, st_grid = _check(g, algo, "grid")
        _, st_auto = _check(g, algo, None)  # the library's choice by size (here the grid)
        for k in keys:
            assert st_wg[k] == st_grid[k] == st_auto[k], (algo, k, st_wg[k], st_grid[k], st_auto[k])
        if algo == "peelone":
            for st in (st_wg, st_grid, st_auto):
                assert 0 < st["pushes_dynamic"] < st["frontier_total"]
            assert st_auto["scans"] == st_grid["scans"]
            assert st_wg["scans"] <= st_grid["scans"] <= st_wg["scans"] + 1


@pytest.mark.parametrize("algo", ALGOS)
def test_large_clique(algo):
    g = gg.complete(2000)
    got = _run(g, algo)
    assert (got == 1999).all()


@pytest.mark.parametrize("algo", ALGOS)
def test_long_path(algo):
    g = gg.path(200_000)
    got = _run(g, algo)
    assert (got == 1).all()


@pytest.mark.parametrize("blocks", [1, 3, 7, 13, 100])
def test_grid_path_any_grid_size(blocks, monkeypatch):
    """The persistent kernels are correct on any grid, including fewer
    workgroups than barrier groups (the library picks small grids for small
    graphs; PICO_GRID_BLOCKS forces one)."""
    monkeypatch.setenv("PICO_GRID_BLOCKS", str(blocks))
    g = gg.rmat(13, 16, 17)
    print(f"case {g.name} n={g.n} m={g.m} blocks={blocks}", flush=True)
    for algo in ALGOS:
        _check(g, algo, "grid")


@pytest.mark.parametrize("path", [None, "grid"])
def test_er10k_both_and_schedules(path):
    g = gg.er_10k()
    want, st_po = _check(g, "peelone", path)
    levels = len(np.unique(want[want > 0]))
    assert st_po["iterations"] == levels
    assert st_po["frontier_total"] == int((want > 0).sum())
    assert st_po["k_max"] == int(want.max())
    _, st_hc = _check(g, "histocore", path)
    _, per_round, _ = oracle.hindex_jacobi(g.offsets, g.cols)
    assert st_hc["iterations"] == len(per_round)
    assert st_hc["frontier_total"] == sum(per_round)


def _schedule(g, algo):
    """(coreness, stats, steps) of the grid path with the per-step record."""
    d = _gpu(g)
    core, st, steps = pico.coreness_schedule(d.offsets, d.cols, algo)
    torch.cuda.synchronize()
    return core.cpu().numpy(), st, steps.numpy()


def _check_peelone_levels(want, st, steps):
    """PeelOne's levels are the distinct non-zero coreness values in
    increasing order, and level k peels exactly {v : core(v) = k} (Alg. 4,
    Table V: l1 = k_max when no level is empty)."""
    vals, counts = np.unique(want[want > 0], return_counts=True)
    assert steps.shape[0] == st["iterations"] == vals.size
    assert np.array_equal(steps[:, 0], vals), "levels visited differ from the coreness values"
    assert np.array_equal(steps[:, 1], counts), "vertices peeled per level differ"
    assert (steps[:, 2] > 0).all() and (steps[:, 4] >= 0).all() and (steps[:, 7] == 0).all()


def _check_histocore_rounds(st, steps, per_round, m):
    """HistoCore's round-t frontier is the synchronous iteration's round-t
    changed set (Theorem 2): sizes compared round by round.  Rounds that
    rebuilt the histograms (kind 1) read all m entries and move nothing."""
    assert steps.shape[0] == st["iterations"] == len(per_round)
    assert np.array_equal(steps[:, 0], np.arange(1, len(per_round) + 1))
    assert np.array_equal(steps[:, 1], np.asarray(per_round, dtype=np.int64)), \
        f"frontier sizes {steps[:, 1].tolist()} vs synchronous rounds {list(per_round)}"
    kind = steps[:, 7]
    assert set(kind.tolist()) <= {0, 1} and int((kind == 1).sum()) == st["scans"]
    assert int(steps[kind == 0, 3].sum()) + m * int((kind == 1).sum()) == st["edges_scanned"]
    assert int(steps[:, 2].sum()) == st["atomics"]  # histogram moves, round by round
    assert (steps[kind == 1, 2] == 0).all()
    assert (steps[:, 4] == 1).all()


@pytest.mark.parametrize("local_edges", ["0", "1", "300", "100000"])
def test_peelone_local_expansion_bound(local_edges, monkeypatch):
    """PeelOne's bound on workgroup-local expansion (PICO_PO_LOCAL_EDGES; 0:
    every asserted vertex waits for the next shared round) moves work between
    the LDS continuation queue and the global rounds, never the result: the
    coreness and the level-by-level schedule equal BZ's."""
    monkeypatch.setenv("PICO_PO_LOCAL_EDGES", local_edges)
    g = gg.scaled_rmat_block(14, 7, 300, 0.6, 40)
    print(f"case {g.name} n={g.n} m={g.m} local_edges={local_edges}", flush=True)
    want = oracle.bz_coreness(g.offsets, g.cols)
    core, st, steps = _schedule(g, "peelone")
    assert np.array_equal(core, want)
    _check_peelone_levels(want, st, steps)
    if local_edges == "0":
        assert st["sub_rounds"] > 0  # the asserted vertices went through shared rounds


@pytest.mark.parametrize("make", [lambda: gg.er_10k(), lambda: gg.rmat(13, 16, 8),
                                  lambda: gg.scaled_rmat_block(14, 7, 300, 0.6, 40),
                                  lambda: gg.disjoint_union(gg.complete(30), gg.cycle(50), gg.empty_graph(4))])
def test_schedule_matches_oracle_per_step(make):
    """The per-step schedule against the oracle, element by element: PeelOne
    level by level against BZ's coreness, HistoCore round by round against
    the synchronous h-index iteration (hindex_jacobi)."""
    g = make()
    print(f"case {g.name} n={g.n} m={g.m}", flush=True)
    want = oracle.bz_coreness(g.offsets, g.cols)
    core, st, steps = _schedule(g, "peelone")
    assert np.array_equal(core, want)
    _check_peelone_levels(want, st, steps)
    core, st, steps = _schedule(g, "histocore")
    assert np.array_equal(core, want)
    _, per_round, _ = oracle.hindex_jacobi(g.offsets, g.cols)
    _check_histocore_rounds(st, steps, per_round, g.m)


@pytest.mark.parametrize("make", [lambda: gg.er_gnp(1500, 6.0, 4), lambda: gg.rmat(10, 8, 2), lambda: gg.g1()])
def test_schedule_matches_serial_traces(make):
    """On small graphs the serial Alg. 4 / Alg. 6 traces give the sets
    themselves: PeelOne's level k holds the trace's scan plus dynamic
    frontier of level k; HistoCore's round t has the trace's V_cnt, whose
    degrees sum to the round's UpdateHisto edge space."""
    g = make()
    deg = np.diff(g.offsets.numpy().astype(np.int64))
    core, st, steps = _schedule(g, "peelone")
    tr = oracle.peelone_trace(g.offsets, g.cols)
    lv = [(L["k"], len(L["scan"]) + len(L["dynamic"])) for L in tr["levels"] if L["scan"] or L["dynamic"]]
    assert [tuple(r) for r in steps[:, :2].tolist()] == lv
    core, st, steps = _schedule(g, "histocore")
    ht = oracle.histocore_trace(g.offsets, g.cols)
    assert steps[:, 1].tolist() == [len(f) for f in ht["frontiers"]]
    assert steps[:, 3].tolist() == [int(deg[f].sum()) for f in ht["frontiers"]]


def test_schedule_rmat22_full_size(golden_rmat22_jacobi):
    """RMAT-22 at full size: PeelOne's levels against BZ, HistoCore's 29
    rounds against the synchronous iteration's changed counts stored by
    tests/golden/make_schedules.py (the same graph, checked by fingerprint)."""
    gold = golden_rmat22_jacobi
    g = gg.rmat22(device="cuda")
    print(f"case {g.name} n={g.n} m={g.m}", flush=True)
    off_h, cols_h = g.offsets.cpu().numpy(), g.cols.cpu().numpy()
    assert (g.n, g.m) == (int(gold["n"][0]), int(gold["m"][0]))
    assert fingerprint(off_h, cols_h) == gold["sha256"][0], "not the graph the stored schedule was taken on"
    want = oracle.bz_coreness(off_h, cols_h)
    core, st, steps = pico.coreness_schedule(g.offsets, g.cols, "peelone")
    assert np.array_equal(core.cpu().numpy(), want)
    _check_peelone_levels(want, st, steps.numpy())
    core, st, steps = pico.coreness_schedule(g.offsets, g.cols, "histocore")
    assert np.array_equal(core.cpu().numpy(), want)
    _check_histocore_rounds(st, steps.numpy(), [int(x) for x in gold["changed_per_round"]], g.m)


_REBUILD_CASE = []


def _rebuild_case():
    """An R-MAT graph beside a star of 5,000 leaves (a row above the LDS
    histogram size whose value falls to 1) and K_2100 (rows above it whose
    value stays 2,099), int64 offsets; with the oracle's coreness and
    synchronous rounds, computed once."""
    if not _REBUILD_CASE:
        g = gg.disjoint_union(gg.rmat(13, 16, 41), gg.star(5000), gg.complete(2100)).with_offsets(torch.int64)
        want = oracle.bz_coreness(g.offsets, g.cols)
        _, per_round, _ = oracle.hindex_jacobi(g.offsets, g.cols)
        _REBUILD_CASE.append((g, want, per_round))
    return _REBUILD_CASE[0]


@pytest.mark.parametrize("permille", ["1", "300", "700", "2000"])
def test_rebuild_rounds_keep_the_schedule(permille, monkeypatch):
    """Histogram rebuild rounds in place of UpdateHisto, from every round
    (share 1/1000) to none (2000): the same coreness, rounds and per-round
    frontiers (the synchronous iteration's, Theorem 2); only the work counts
    change.  Includes heavy rows (the planted block's vertices have more than
    2,048 neighbours) and int64 offsets."""
    monkeypatch.setenv("PICO_HC_REBUILD_PERMILLE", permille)
    g, want, per_round = _rebuild_case()
    print(f"case {g.name} n={g.n} m={g.m} permille={permille}", flush=True)
    core, st, steps = _schedule(g, "histocore")
    assert np.array_equal(core, want)
    _check_histocore_rounds(st, steps, per_round, g.m)
    # the rule: a round rebuilds iff its frontier rows hold >= permille / 1000 of m
    want_kind = (steps[:, 3] * 1000 >= int(permille) * g.m).astype(np.int64)
    assert np.array_equal(steps[:, 7], want_kind)
    if permille == "1":
        assert st["scans"] >= 1
    if permille == "2000":
        assert st["scans"] == 0


def test_schedule_cap_and_errors():
    """A short array gets the first cap records and the full count; cap 0
    records nothing; the one-workgroup path and the ablations are refused."""
    g = _gpu(gg.rmat(12, 16, 5))
    a = pico.algo_code("peelone", g.offsets)
    ws = pico.workspace_for(g.n, g.m, a, "cuda")
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    full = torch.zeros((4096, 8), dtype=torch.int64, device="cuda")
    rc, count = pico.pico_coreness_schedule(g.offsets, g.cols, g.n, g.m, a, out, ws, ws.numel(), None, full,
                                            4096)
    assert rc == pico.PICO_OK and 3 < count < 4096
    short = torch.full((3, 8), -9, dtype=torch.int64, device="cuda")
    rc, count2 = pico.pico_coreness_schedule(g.offsets, g.cols, g.n, g.m, a, out, ws, ws.numel(), None, short, 2)
    assert rc == pico.PICO_OK and count2 == count
    s = short.cpu()
    assert torch.equal(s[:2, :2], full[:2, :2].cpu()) and (s[2] == -9).all()
    rc, count3 = pico.pico_coreness_schedule(g.offsets, g.cols, g.n, g.m, a, out, ws, ws.numel(), None, None, 0)
    assert rc == pico.PICO_OK and count3 == count
    for bad in (a | pico.PICO_PATH_WG, a | pico.PICO_PO_GPP, pico.PICO_ALGO_CNTCORE):
        rc, _ = pico.pico_coreness_schedule(g.offsets, g.cols, g.n, g.m, bad, out, ws, ws.numel(), None, full, 8)
        assert rc == pico.PICO_EINVAL


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("offsets_dtype", [torch.int32, torch.int64])
def test_rmat_medium(algo, offsets_dtype):
    g = gg.rmat(16, 16, 3).with_offsets(offsets_dtype)
    print(f"case {g.name} n={g.n} m={g.m} algo={algo} {offsets_dtype}", flush=True)
    _check(g, algo)


@pytest.mark.parametrize("algo", ALGOS)
def test_rmat_block_deep_hierarchy(algo):
    g = gg.scaled_rmat_block(16, 7, 600, 0.6, 70, offsets_dtype=torch.int64)
    print(f"case {g.name} n={g.n} m={g.m}", flush=True)
    _check(g, algo)


@pytest.mark.parametrize("path", ["grid", "wg"])
def test_histocore_rounds_match_jacobi_both_paths(path):
    """Round count and total frontier on either path (the one-workgroup path
    keeps no per-round record; the grid path's record is compared round by
    round in test_schedule_matches_oracle_per_step)."""
    g = gg.rmat(13, 16, 8)
    _, per_round, _ = oracle.hindex_jacobi(g.offsets, g.cols)
    _, st = _check(g, "histocore", path)
    assert st["iterations"] == len(per_round)
    assert st["frontier_total"] == sum(per_round)


@pytest.mark.parametrize("algo", ALGOS)
def test_deterministic_and_relabel_invariant(algo):
    g = gg.rmat(15, 16, 11)
    a = _run(g, algo)
    for _ in range(3):
        assert np.array_equal(a, _run(g, algo))
    # relabel vertices by a bijection: coreness moves with the vertex
    perm = gg.permute_pow2(torch.arange(g.n), 15, 5)
    s, d = g.edge_pairs()
    h = gg.csr_from_pairs(g.n, perm[s], perm[d])
    b = _run(h, algo)
    assert np.array_equal(b[perm.numpy()], a)


@pytest.mark.parametrize("algo", ALGOS)
def test_workspace_errors(algo):
    g = _gpu(gg.er_gnp(500, 6.0, 2))
    a = pico.algo_code(algo, g.offsets)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    need = pico.pico_workspace_bytes(g.n, g.m, a)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    rc = pico.pico_coreness_ws(g.offsets, g.cols, g.n, g.m, a, out, ws, need - 4096)
    assert rc == pico.PICO_ENOMEM
    rc = pico.pico_coreness_ws(g.offsets, g.cols, g.n, g.m, a, out, ws, need)
    assert rc == pico.PICO_OK
    want = oracle.bz_coreness(g.offsets.cpu(), g.cols.cpu())
    assert np.array_equal(out.cpu().numpy(), want)
    # the self-allocating entry point agrees
    out2 = torch.full_like(out, -7)
    assert pico.pico_coreness(g.offsets, g.cols, g.n, g.m, a, out2) == pico.PICO_OK
    torch.cuda.synchronize()
    assert torch.equal(out, out2)


def test_validate_csr():
    g = _gpu(gg.er_gnp(300, 5.0, 1))
    assert pico.pico_validate_csr(g.offsets, g.cols, g.n, g.m, 0) == pico.PICO_OK
    bad = g.cols.clone()
    bad[3] = g.n + 5
    assert pico.pico_validate_csr(g.offsets, bad, g.n, g.m, 0) == pico.PICO_EBADCSR


@pytest.mark.parametrize("algo", ALGOS)
def test_rmat22_full_size(algo):
    """The RMAT-22 workload at full size, against the oracle on every vertex."""
    g = gg.rmat22(device="cuda")
    print(f"case {g.name} n={g.n} m={g.m} algo={algo}", flush=True)
    got = pico.coreness(g.offsets, g.cols, algo).cpu().numpy()
    want = oracle.bz_coreness(g.offsets.cpu(), g.cols.cpu())
    assert np.array_equal(got, want)


def test_rmat26_block_full_size():
    """The RMAT-26 + planted-block workload at full size (int64 offsets, m of
    2.1 billion), in the launch configuration bench.py times: both algorithms
    against the oracle (BZ on the host over the whole graph) on every vertex;
    PeelOne's level count and k_max against the oracle's coreness; the
    properties that hold at any size as an extra."""
    import bench
    g = gg.rmat26_block(device="cuda")
    print(f"case {g.name} n={g.n} m={g.m}", flush=True)
    assert g.offsets.dtype == torch.int64 and g.m > 2 ** 30
    po, st_po = pico.coreness(g.offsets, g.cols, "peelone", with_stats=True)
    hc, st_hc = pico.coreness(g.offsets, g.cols, "histocore", with_stats=True)
    props = bench.coreness_properties(g.offsets, g.cols, po)
    assert all(props.values()), props
    po, hc = po.cpu().numpy(), hc.cpu().numpy()
    off_h = g.offsets.cpu().numpy()
    cols_h = g.cols.cpu().numpy()
    del g
    torch.cuda.empty_cache()
    print("oracle: BZ over the whole graph", flush=True)
    want = oracle.bz_coreness(off_h, cols_h)
    for name, got in (("peelone", po), ("histocore", hc)):
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, f"{name}: {bad.size} vertices differ from the oracle, first {bad[:5]}"
    vals = np.unique(want[want > 0])
    assert st_po["iterations"] == vals.size
    assert st_po["k_max"] == int(want.max())
    assert st_po["frontier_total"] == int((want > 0).sum())
