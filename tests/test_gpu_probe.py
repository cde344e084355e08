"""GPU random-access probe (pico_probe_random_access): the measurement aid
the bench sets the kernels' times against.  Only sanity is checkable: both
rates positive and finite, and the call leaves the device usable."""
import math

import pytest
import torch

import paper_2402_15253_amd as pico

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [4, 1 << 20, 64 << 20])
def test_probe_rates(nbytes):
    r = pico.probe_random_access(nbytes, ops=1 << 20)
    assert r["bytes"] == nbytes
    for k in ("gathers_per_s", "atomics_per_s"):
        assert math.isfinite(r[k]) and r[k] > 0, r
    # the device still decomposes a graph correctly afterwards
    off = torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda")
    cols = torch.tensor([1, 0], dtype=torch.int32, device="cuda")
    assert pico.coreness(off, cols, "peelone").cpu().tolist() == [1, 1]
