"""pico_coreness_noalloc (workspace in the library's static device array, no
allocation during the call) against pico_coreness (stream-ordered allocation)
through the C ABI: bit-exact on consecutive calls that shrink, on both the
grid and the one-workgroup path, with int32 and int64 offsets."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_2402_15253_amd as pico

pytestmark = pytest.mark.gpu


def _calls(algo, graphs):
    for g in graphs:
        print(f"case {g.name} n={g.n} m={g.m} algo={algo} {g.offsets.dtype}", flush=True)
        a = pico.algo_code(algo, g.offsets)
        assert pico.pico_workspace_bytes(g.n, g.m, a) <= pico.PICO_NOALLOC_SCRATCH_BYTES
        ref = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
        assert pico.pico_coreness(g.offsets, g.cols, g.n, g.m, a, ref) == pico.PICO_OK, pico.pico_last_error()
        out = torch.full((g.n,), -9, dtype=torch.int32, device="cuda")
        rc = pico.pico_coreness_noalloc(g.offsets, g.cols, g.n, g.m, a, out)
        assert rc == pico.PICO_OK, pico.pico_last_error()
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        want = oracle.bz_coreness(g.offsets.cpu(), g.cols.cpu())
        assert np.array_equal(out.cpu().numpy(), want)


@pytest.mark.parametrize("algo", ["peelone", "histocore"])
@pytest.mark.parametrize("offsets_dtype", [torch.int32, torch.int64])
def test_noalloc_matches_pico_coreness_on_shrinking_calls(algo, offsets_dtype):
    graphs = [gg.rmat(15, 16, 31), gg.er_gnp(3000, 8.0, 7), gg.er_gnp(600, 6.0, 3)]
    _calls(algo, [g.with_offsets(offsets_dtype).to("cuda") for g in graphs])


def test_noalloc_refuses_a_graph_beyond_its_scratch():
    g = gg.rmat(15, 16, 31).to("cuda")
    a = pico.algo_code("histocore", g.offsets)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    rc = pico.pico_coreness_noalloc(g.offsets, g.cols, 20_000_000, g.m, a, out)  # claims 20M vertices
    assert rc == pico.PICO_ENOMEM and "static scratch" in pico.pico_last_error()
    # the array is still usable afterwards
    _calls("histocore", [gg.er_gnp(2000, 5.0, 9).to("cuda")])
