"""GPU parity of the batched entry point: every graph of a packed batch gets
exactly the oracle's coreness, and the same result as a plain single-graph
call, whether its values live in LDS or in global memory."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_2402_15253_amd as pico

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    b = gg.mixed_batch(64, 2, 60_000, seed=31)
    # add edge cases: empty graphs, a clique, a star, a path
    return b


def _per_graph_oracle(b):
    return [oracle.bz_coreness(*(lambda g: (g.offsets, g.cols))(b.graph(g)))
            for g in range(b.num_graphs)]


@pytest.mark.parametrize("algo", ["peelone", "histocore"])
@pytest.mark.parametrize("lds_bytes", [-1, 0])
def test_batched_matches_oracle(batch, algo, lds_bytes):
    want = np.concatenate(_per_graph_oracle(batch))
    d = batch.to("cuda")
    tune = pico.BatchTune(lds_bytes, 0)
    got, st = pico.coreness_batched(d, algo, tune=tune, with_stats=True)
    got = got.cpu().numpy()
    print(f"{algo} lds_bytes={lds_bytes} stats={st}", flush=True)
    assert np.array_equal(got, want)
    if lds_bytes == 0:
        assert st["lds_graphs"] == 0
    else:
        assert st["lds_graphs"] > 0


def test_batched_equals_plain_calls(batch):
    d = batch.to("cuda")
    got = pico.coreness_batched(d, "peelone")
    torch.cuda.synchronize()
    for g in range(0, batch.num_graphs, 7):
        x0, x1 = int(batch.vptr[g]), int(batch.vptr[g + 1])
        one = batch.graph(g).to("cuda")
        if one.n == 0:
            continue
        plain = pico.coreness(one.offsets, one.cols, "histocore")
        assert torch.equal(plain, got[x0:x1])


def test_batched_edge_cases():
    parts = [gg.empty_graph(0), gg.empty_graph(5), gg.complete(30), gg.star(300), gg.path(1000),
             gg.g1(), gg.hypercube(7)]
    srcs, dsts, sizes, base = [], [], [], 0
    for p in parts:
        s, t = p.edge_pairs()
        srcs.append(s + base)
        dsts.append(t + base)
        sizes.append(p.n)
        base += p.n
    b = gg.pack_pairs(torch.tensor(sizes), torch.cat(srcs), torch.cat(dsts), name="edge-cases")
    want = np.concatenate([oracle.bz_coreness(p.offsets, p.cols) for p in parts])
    d = b.to("cuda")
    for algo in ("peelone", "histocore"):
        got = pico.coreness_batched(d, algo).cpu().numpy()
        assert np.array_equal(got, want), algo


@pytest.mark.parametrize("lds_bytes", [0, -1])
def test_batched_peelone_with_helpers(batch, lds_bytes):
    """PeelOne graphs above a (here small) vertex count are decomposed by
    their workgroup with idle workgroups claiming chunks of each phase; the
    result is the oracle's either way."""
    _helped_batch(batch, lds_bytes, "peelone")


@pytest.mark.parametrize("lds_bytes", [0, -1])
def test_batched_histocore_with_helpers(batch, lds_bytes):
    """The same for HistoCore: set-up, SumHisto and UpdateHisto phases shared
    out, rounds still synchronous."""
    _helped_batch(batch, lds_bytes, "histocore")


def _helped_batch(batch, lds_bytes, algo):
    want = np.concatenate(_per_graph_oracle(batch))
    d = batch.to("cuda")
    tune = pico.BatchTune(lds_bytes, 0, 0, 1000)
    got, st = pico.coreness_batched(d, algo, tune=tune, with_stats=True)
    print(f"helpers lds_bytes={lds_bytes} stats={st}", flush=True)
    assert np.array_equal(got.cpu().numpy(), want)
    assert st["helped_graphs"] > 0


def test_few_large_graphs_mostly_helped():
    """Three large graphs in a launch of hundreds of workgroups: nearly all
    of them help, and every phase's chunks are shared out."""
    parts = [gg.rmat(15, 16, 41), gg.er_gnp(20_000, 10.0, 42), gg.scaled_rmat_block(14, 43, 200, 0.6, 44)]
    srcs, dsts, sizes, base = [], [], [], 0
    for p in parts:
        s, t = p.edge_pairs()
        srcs.append(s + base)
        dsts.append(t + base)
        sizes.append(p.n)
        base += p.n
    b = gg.pack_pairs(torch.tensor(sizes), torch.cat(srcs), torch.cat(dsts), name="three-large")
    want = np.concatenate([oracle.bz_coreness(p.offsets, p.cols) for p in parts])
    d = b.to("cuda")
    for algo in ("peelone", "histocore"):
        for help_min in (1000, -1):
            got, st = pico.coreness_batched(d, algo, tune=pico.BatchTune(0, 0, 0, help_min),
                                            with_stats=True)
            print(f"{algo} help_min={help_min} stats={st}", flush=True)
            assert np.array_equal(got.cpu().numpy(), want), (algo, help_min)
            if help_min > 0:
                assert st["helped_graphs"] == 3 and st["help_chunks"] > 0
            else:
                assert st["helped_graphs"] == 0


def _pack(parts, name):
    srcs, dsts, sizes, base = [], [], [], 0
    for p in parts:
        s, t = p.edge_pairs()
        srcs.append(s + base)
        dsts.append(t + base)
        sizes.append(p.n)
        base += p.n
    return gg.pack_pairs(torch.tensor(sizes), torch.cat(srcs), torch.cat(dsts), name=name)


def _auto_parts():
    """Graphs whose first frontier is empty (every vertex has as many
    neighbours of degree >= its own as its degree: a union of cliques of 30
    sizes, a hypercube, a cycle) between skewed and random ones."""
    hc = [gg.disjoint_union(*[gg.complete(k) for k in range(3, 33)]), gg.hypercube(9), gg.cycle(700)]
    po = [gg.rmat(12, 16, 5), gg.er_gnp(3000, 8.0, 6), gg.rmat(10, 8, 7), gg.scaled_rmat_block(12, 8, 150, 0.7, 9)]
    parts = [po[0], hc[0], po[1], hc[1], po[2], hc[2], po[3]]
    return parts, [1, 3, 5]


@pytest.mark.parametrize("lds_bytes", [-1, 0])
def test_batched_auto_chooses_per_graph(lds_bytes):
    """PICO_ALGO_AUTO: the graphs whose sampled first frontier is empty go to
    HistoCore, the rest to PeelOne; every graph gets the oracle's coreness
    and every status word reads PICO_OK."""
    parts, hc_idx = _auto_parts()
    b = _pack(parts, "auto-mix")
    want = np.concatenate([oracle.bz_coreness(p.offsets, p.cols) for p in parts])
    d = b.to("cuda")
    got, st = pico.coreness_batched(d, "auto", tune=pico.BatchTune(lds_bytes, 0), with_stats=True)
    print(f"auto lds_bytes={lds_bytes} stats={st}", flush=True)
    assert np.array_equal(got.cpu().numpy(), want)
    assert st["histocore_graphs"] == len(hc_idx) and st["graphs"] == len(parts)


def test_batch_status_after_enqueue_only(batch):
    """Without stats the call only enqueues; pico_batch_status then waits and
    reports one word per graph: all PICO_OK, and the results are the
    oracle's.  Also under PICO_ALGO_AUTO."""
    want = np.concatenate(_per_graph_oracle(batch))
    d = batch.to("cuda")
    G, n, m = batch.num_graphs, d.offsets.numel() - 1, d.cols.numel()
    for algo in ("peelone", "auto"):
        code = pico.BATCH_ALGOS[algo]
        wsb = pico.pico_batched_workspace_bytes(G, n, m, code)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        out = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        rc = pico.pico_coreness_batched(d.vptr, d.offsets, d.cols, G, n, m, code, None, out, None, ws, wsb)
        assert rc == pico.PICO_OK, pico.pico_last_error()
        rc, words = pico.batch_status(ws, G)
        assert rc == pico.PICO_OK and words.shape == (G,) and (words == 0).all(), (algo, words)
        assert np.array_equal(out.cpu().numpy(), want), algo


@pytest.mark.parametrize("algo", ["peelone", "histocore"])
def test_tiny_wait_bound_reports_unfinished_graphs(algo, monkeypatch):
    """Every wait of the batched kernel given up after about a microsecond
    (PICO_BATCH_WAIT_US): helpers leave almost at once, and a leader still
    waiting for a helper's chunk gives up, leaves its graph unfinished and
    takes no other graph.  Every kernel still ends; each graph's status word
    reads PICO_OK (and its result is the oracle's) or PICO_EHIP, and the call
    with stats returns PICO_EHIP exactly when some word does."""
    monkeypatch.setenv("PICO_BATCH_WAIT_US", "1")
    parts = [gg.rmat(15, 16, 41), gg.er_gnp(20_000, 10.0, 42), gg.scaled_rmat_block(14, 43, 200, 0.6, 44),
             gg.er_gnp(3000, 6.0, 45), gg.rmat(11, 8, 46)]
    b = _pack(parts, "tiny-wait")
    wants = [oracle.bz_coreness(p.offsets, p.cols) for p in parts]
    d = b.to("cuda")
    G, n, m = b.num_graphs, d.offsets.numel() - 1, d.cols.numel()
    code = pico.BATCH_ALGOS[algo]
    wsb = pico.pico_batched_workspace_bytes(G, n, m, code)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    out = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    st = pico.BatchStats()
    rc = pico.pico_coreness_batched(d.vptr, d.offsets, d.cols, G, n, m, code, None, out,
                                    pico.BatchTune(0, 0, 0, 1000), ws, wsb, st)
    rc2, words = pico.batch_status(ws, G)
    print(f"{algo}: call {rc} status {rc2} words {words.tolist()} stats {st.as_dict()}", flush=True)
    assert set(words.tolist()) <= {pico.PICO_OK, pico.PICO_EHIP}
    assert rc == rc2 == (pico.PICO_EHIP if (words != 0).any() else pico.PICO_OK)
    got = out.cpu().numpy()
    vp = b.vptr.numpy()
    for g in range(G):
        if words[g] == pico.PICO_OK:
            assert np.array_equal(got[vp[g]:vp[g + 1]], wants[g]), g


def test_autotuned_launch_on_every_size_class(tmp_path, monkeypatch):
    """The autotuner's chosen launch (timed afresh: the cache points to an
    empty file) on a batch that reaches the largest size class -- graphs of
    up to 200,000 vertices, above the LDS tier and above the helpers'
    threshold -- against the oracle on every graph, for both algorithms and
    the per-graph choice."""
    from paper_2402_15253_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    b = gg.mixed_batch(48, 200, 200_000, seed=4096)
    sizes = (b.vptr[1:] - b.vptr[:-1]).numpy()
    assert sizes.max() > 65_536 and sizes.min() < 4096
    want = np.concatenate(_per_graph_oracle(b))
    d = b.to("cuda")
    order = pico.largest_first(d.vptr)
    for algo in ("peelone", "histocore", "auto"):
        tune = autotune.tune_batched(d, algo, order=order, use_cache=True)
        got, st = pico.coreness_batched(d, algo, tune=tune, order=order, with_stats=True)
        print(f"{algo} tune={tune.as_dict()} stats={st}", flush=True)
        assert np.array_equal(got.cpu().numpy(), want), algo
        assert st["lds_graphs"] < b.num_graphs
