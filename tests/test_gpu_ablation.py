"""GPU PeelOne ablations (PICO_PO_STATIC, PICO_PO_ROLLBACK, PICO_PO_GPP)
against the oracle.

Both give the coreness bit for bit.  Without the dynamic frontier the
iteration count is fixed by the graph (every scan sees the values the
previous iteration left), and it must equal the serial oracle's
(``oracle.peel_static``), including the closed form for a path and G1's
narrative; the dynamic run needs one level per distinct coreness value
(Table V), so the gap is what the dynamic frontier saves (Table IV vs V).
The rollback decrement issues at least as many atomics as it has
decrements, plus one per undone decrement."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_2402_15253_amd as pico

pytestmark = pytest.mark.gpu

GRAPHS = [lambda: gg.g1(), lambda: gg.path(1001), lambda: gg.star(3000), lambda: gg.rmat(12, 16, 71),
          lambda: gg.er_gnp(4000, 8.0, 72), lambda: gg.rmat(14, 16, 73).with_offsets(torch.int64),
          lambda: gg.scaled_rmat_block(13, 74, 300, 0.6, 75)]


def _run(g, algo):
    d = g.to("cuda")
    got, st = pico.coreness(d.offsets, d.cols, algo, with_stats=True)
    torch.cuda.synchronize()
    return got.cpu().numpy(), st


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_static_matches_serial_schedule(gi):
    g = GRAPHS[gi]()
    print(f"case {g.name} n={g.n} m={g.m}", flush=True)
    want, iters = oracle.peel_static(g.offsets, g.cols)
    assert np.array_equal(want, oracle.bz_coreness(g.offsets, g.cols))
    got, st = _run(g, "peelone-static")
    assert np.array_equal(got, want)
    assert st["iterations"] == iters
    assert st["pushes_dynamic"] == 0
    _, st_dyn = _run(g, "peelone")
    assert st_dyn["iterations"] == len(np.unique(want[want > 0])) <= iters


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_rollback_matches_oracle(gi):
    g = GRAPHS[gi]()
    print(f"case {g.name} n={g.n} m={g.m}", flush=True)
    want = oracle.bz_coreness(g.offsets, g.cols)
    got, st = _run(g, "peelone-rollback")
    assert np.array_equal(got, want)
    _, st_dyn = _run(g, "peelone")
    assert st["iterations"] == st_dyn["iterations"]
    assert st["frontier_total"] == int((want > 0).sum())


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_gpp_matches_serial_schedule(gi):
    """General Parallel Peel (Alg. 3): same coreness; its while-loop
    iterations (k raised at the head of an iteration when nobody residual is
    at or below it) are fixed by the graph and equal the serial oracle's, and
    so is its decrement count: every removed vertex decrements each neighbour
    still residual, one atomic per such edge."""
    g = GRAPHS[gi]()
    print(f"case {g.name} n={g.n} m={g.m}", flush=True)
    want, iters, decrements = oracle.peel_gpp(g.offsets, g.cols)
    assert np.array_equal(want, oracle.bz_coreness(g.offsets, g.cols))
    got, st = _run(g, "gpp")
    assert np.array_equal(got, want)
    assert st["iterations"] == iters
    assert st["atomics"] == decrements  # removal flags are set before the decrements run
    assert st["pushes_dynamic"] == 0
