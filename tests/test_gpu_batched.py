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
