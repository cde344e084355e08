"""GPU core maintenance (pico_coreness_update): HistoCore started from upper
bounds of the coreness, against the oracle on the changed graph.

Bit-exact coreness against BZ on the new graph; the round count and per-round
frontier sizes equal the oracle's iteration from the same bounds (the
synchronous rounds of Theorem 2, started from the bounds instead of the
degrees)."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_2402_15253_amd as pico

pytestmark = pytest.mark.gpu

GRAPHS = [lambda: gg.rmat(12, 16, 31), lambda: gg.er_gnp(5000, 8.0, 32), lambda: gg.rmat(15, 16, 33)]


def _update(h, prev, add, path=None, out=None):
    d = h.to("cuda")
    p = torch.from_numpy(np.ascontiguousarray(prev)).to("cuda")
    got, st = pico.coreness_update(d.offsets, d.cols, p, add, with_stats=True, path=path,
                                   out=p if out == "inplace" else None)
    torch.cuda.synchronize()
    return got.cpu().numpy(), st


@pytest.mark.parametrize("path", [None, "grid", "wg"])
@pytest.mark.parametrize("gi", range(len(GRAPHS)))
@pytest.mark.parametrize("edit", ["delete", "insert"])
def test_update_matches_oracle(gi, edit, path):
    g = GRAPHS[gi]()
    if path == "wg" and g.n > 30000:
        pytest.skip("values do not fit one workgroup's LDS")
    old = oracle.bz_coreness(g.offsets, g.cols)
    h, b = gg.edit_edges(g, 0.03, 0 if edit == "delete" else 40, 7 + gi)
    print(f"case {h.name} n={h.n} m={h.m} b={b} path={path}", flush=True)
    want = oracle.bz_coreness(h.offsets, h.cols)
    got, st = _update(h, old, b, path)
    mism = np.nonzero(got != want)[0]
    assert mism.size == 0, f"{mism.size} mismatches, first {mism[:5]} got {got[mism[:5]]} want {want[mism[:5]]}"
    _, per_round, _ = oracle.hindex_jacobi_from(h.offsets, h.cols, old, add=b)
    assert st["iterations"] == len(per_round)
    assert st["frontier_total"] == sum(per_round)


@pytest.mark.parametrize("offsets_dtype", [torch.int32, torch.int64])
def test_update_in_place_and_fewer_rounds(offsets_dtype):
    g = gg.rmat(16, 16, 34).with_offsets(offsets_dtype)
    d = g.to("cuda")
    old = pico.coreness(d.offsets, d.cols, "peelone")
    h, _ = gg.edit_edges(g, 0.01, 0, 35)
    h = h.with_offsets(offsets_dtype)
    e = h.to("cuda")
    want, st_cold = pico.coreness(e.offsets, e.cols, "histocore", with_stats=True)
    prev = old.clone()
    got, st = pico.coreness_update(e.offsets, e.cols, prev, 0, out=prev, with_stats=True)
    torch.cuda.synchronize()
    assert got.data_ptr() == prev.data_ptr()
    assert torch.equal(got, want)
    assert torch.equal(want, pico.coreness(e.offsets, e.cols, "peelone"))
    assert st["iterations"] <= st_cold["iterations"]
    assert st["frontier_total"] < st_cold["frontier_total"]


def test_update_from_coreness_is_a_fixed_point():
    g = gg.rmat(14, 16, 36)
    d = g.to("cuda")
    core = pico.coreness(d.offsets, d.cols, "peelone")
    got, st = pico.coreness_update(d.offsets, d.cols, core, 0, with_stats=True)
    assert torch.equal(got, core)
    assert st["iterations"] == 0 and st["frontier_total"] == 0
