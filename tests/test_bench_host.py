"""Host-side arithmetic of bench.py (no GPU): the random-access roofline and
the algorithmic byte models it reports."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


class FakeProbe:
    """Stands in for the library: fixed rates per array size."""

    def __init__(self, rates):
        self.rates = rates
        self.calls = []

    def probe_random_access(self, nbytes, ops):
        self.calls.append(nbytes)
        g, a = self.rates[nbytes]
        return {"bytes": nbytes, "ops": ops, "gathers_per_s": g, "atomics_per_s": a}


def test_random_access_roof_arithmetic():
    n, m = 1000, 8000
    fake = FakeProbe({4 * n: (80e9, 25e9), 4 * m: (50e9, 20e9)})
    st = {"peelone": {"atomics": 3000}, "histocore": {"atomics": 5000, "scans": 2}}
    per_kernel = {"po_persistent": {"avg_ms": 0.5}, "hc_persistent": {"avg_ms": 2.0}}
    r = bench.random_access_roof(fake, st, n, m, per_kernel, ops=1 << 10)
    assert fake.calls == [4 * n, 4 * m]
    po = r["po_persistent"]
    want_po = (m / 80e9 + 3000 / 25e9) * 1e3
    assert po["gathers"] == m and po["atomics"] == 3000
    assert abs(po["ms_at_probe_rates"] - round(want_po, 3)) < 1e-9
    assert abs(po["frac"] - round(want_po / 0.5, 4)) < 1e-9
    hc = r["hc_persistent"]
    # a value gather per entry in InitHisto and in each of the 2 rebuild rounds
    # (value-array rates), two atomics per histogram move (histogram-sized array)
    want_hc = (3 * m / 80e9 + 2 * 5000 / 20e9) * 1e3
    assert hc["atomics"] == 10000 and hc["gathers"] == 3 * m
    assert abs(hc["frac"] - round(want_hc / 2.0, 4)) < 1e-9


def test_random_access_roof_skips_kernels_not_run():
    fake = FakeProbe({40: (1e9, 1e9), 400: (1e9, 1e9)})
    r = bench.random_access_roof(fake, {"peelone": {"atomics": 1}}, 10, 100,
                                 {"po_persistent": {"avg_ms": 1.0}}, ops=8)
    assert "hc_persistent" not in r and "po_persistent" in r


def test_peelone_byte_model():
    # n(2W + 20) + 8m + 8A (per vertex: two offsets, init, scan, queue, output;
    # per entry: column and neighbour value; per decrement: one RMW)
    n, m, w, a = 100, 600, 4, 250
    assert bench.algorithmic_bytes("peelone", {"atomics": a}, n, m, w) == n * (2 * w + 20) + 8 * m + 8 * a


def test_histocore_byte_model_with_rebuild_rounds():
    # a rebuild round replaces UpdateHisto's 8 per scanned entry and 16 per
    # move by InitHisto's n(2W + 4) + 12m over the current values
    n, m, w = 100, 600, 8
    base = {"frontier_total": 70, "pushes_dynamic": 20, "buckets_scanned": 300, "edges_scanned": 900,
            "atomics": 150, "scans": 0}
    b0 = bench.algorithmic_bytes("histocore", base, n, m, w)
    want0 = (n * (2 * w + 8) + 12 * m + 4 * 50) + (70 * (28 + 2 * w) + 4 * 300 + 8 * 900 + 16 * 150 + 4 * 20) + 4 * n
    assert b0 == want0
    reb = dict(base, scans=2, edges_scanned=900 + 2 * m)
    assert bench.algorithmic_bytes("histocore", reb, n, m, w) == want0 + 2 * (n * (2 * w + 4) + 12 * m)


def test_autotune_key_names_kernel_revision(monkeypatch):
    """The batched autotuner's cache key carries the kernel's source hash, so
    a choice timed on another revision of the kernel is not reused."""
    import types

    import torch

    import paper_2402_15253_amd.autotune as at
    from paper_2402_15253_amd.profiling import source_hash

    props = types.SimpleNamespace(name="gfx950", multi_processor_count=256)
    monkeypatch.setattr(torch.cuda, "get_device_properties", lambda dev: props)
    batch = types.SimpleNamespace(offsets=torch.zeros(101, dtype=torch.int64),
                                  cols=torch.zeros(800, dtype=torch.int32),
                                  vptr=torch.zeros(5, dtype=torch.int64))
    key = at._key(batch, "peelone")
    assert key.startswith("gfx950|256|peelone|G4|n25|m2e+02|")
    assert key.endswith(source_hash("batched_kernel"))


def test_code_hash_ignores_comments_not_code():
    """A profile summary stays matched to its kernel through comment and layout
    edits, and stops matching at any change to the code."""
    from paper_2402_15253_amd.profiling import code_hash

    base = code_hash([("k.hip", "int f(int x) { return x + 1; }  // add one\n")])
    assert base == code_hash([("k.hip", "/* add\n   one */\nint f(int x)\n{\n    return x + 1;\n}\n")])
    assert base != code_hash([("k.hip", "int f(int x) { return x + 2; }  // add one\n")])
    assert base != code_hash([("j.hip", "int f(int x) { return x + 1; }")])
