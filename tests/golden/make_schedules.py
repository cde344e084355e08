"""Writes tests/golden/rmat22_jacobi.txt: the per-round changed counts of the
synchronous h-index iteration (Section II-A, Alg. 2 in synchronous rounds) on
the RMAT-22 workload, from the oracle alone.  By Theorem 2 HistoCore's
round-t frontier is exactly round t's changed set, so the GPU schedule test
compares its per-round frontier sizes with these counts.  The iteration
recomputes every h-index by sorting each round, which takes minutes at this
size, hence the stored values.  A fingerprint of the graph (n, m, SHA-256 of
the offsets and column arrays) is stored beside them so the test can check it
decomposes the same graph.

Run from the repository root: python tests/golden/make_schedules.py
"""
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402


def fingerprint(offsets, cols) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(np.asarray(offsets)).tobytes())
    h.update(np.ascontiguousarray(np.asarray(cols)).tobytes())
    return h.hexdigest()


def main():
    g = gg.rmat22(device="cpu")
    off, cols = g.offsets.numpy(), g.cols.numpy()
    x, per_round, _ = oracle.hindex_jacobi(off, cols)
    core = oracle.bz_coreness(off, cols)
    assert np.array_equal(x, core), "the iteration did not reach the coreness"
    path = os.path.join(ROOT, "tests", "golden", "rmat22_jacobi.txt")
    with open(path, "w") as f:
        f.write("# RMAT-22 workload (graphgen.rmat22: scale 22, edge factor 16, seed 22, int32 CSR)\n")
        f.write("# written by tests/golden/make_schedules.py from oracle.hindex_jacobi and oracle.bz_coreness\n")
        f.write(f"n = {g.n}\n")
        f.write(f"m = {g.m}\n")
        f.write(f"sha256 = {fingerprint(off, cols)}\n")
        f.write(f"offsets_dtype = {off.dtype}\n")
        f.write("# vertices whose value changes in synchronous round t = 1, 2, ... (Theorem 2)\n")
        f.write("changed_per_round = " + " ".join(str(int(c)) for c in per_round) + "\n")
        f.write(f"k_max = {int(core.max())}\n")
    print(f"wrote {path}: {len(per_round)} rounds, k_max {int(core.max())}")


if __name__ == "__main__":
    main()
