"""Host check of the argument behind SumHisto's sliced wave sum (the
kernel's `wave_reverse_sum_wide`): scanning buckets top..1, the answer is
the first b with sum(b..top) >= b; since sum(b..top) - b rises strictly as b
falls, it lies in the first slice (from the top) whose lowest bucket already
meets the test.  This re-derives that search in plain Python -- a first pass
of 64 single buckets, then passes of 64 slices of 8 -- and compares it with
the direct scan (Step II of Fig. 6) on random histograms."""
import numpy as np
import pytest

W, U = 64, 8


def direct(seg, top):
    s = 0
    for b in range(top, 0, -1):
        s += int(seg[b - 1])
        if s >= b:
            return b, s
    return 0, s


def sliced(seg, top):
    carry = 0
    run = carry
    for lane in range(W):  # first pass: bucket top - lane
        b = top - lane
        if b < 1:
            break
        run += int(seg[b - 1])
        if run >= b:
            return b, run
    carry = run
    top -= W
    while top >= 1:
        sums, slices = [], []
        for lane in range(W):
            hi = top - lane * U
            vals = [int(seg[hi - j - 1]) if hi - j >= 1 else 0 for j in range(U)]
            slices.append((hi, vals))
            sums.append(sum(vals))
        prefix = carry
        for lane, (hi, vals) in enumerate(slices):
            prefix += sums[lane]
            lo = max(hi - U + 1, 1)
            if hi >= 1 and prefix >= lo:  # the answer is inside this slice
                r = prefix - sums[lane]
                for j, v in enumerate(vals):
                    r += v
                    if hi - j >= 1 and r >= hi - j:
                        return hi - j, r
                raise AssertionError("slice chosen without an answer")
        carry = prefix
        top -= W * U
    return 0, carry


@pytest.mark.parametrize("seed", range(4))
def test_sliced_search_equals_direct_scan(seed):
    rng = np.random.default_rng(seed)
    for t in range(400):
        top = int(rng.integers(1, 4097))
        kind = t % 4
        if kind == 0:
            seg = rng.integers(0, 3, top)
        elif kind == 1:
            seg = (rng.random(top) < 0.05) * rng.integers(1, 50, top)
        elif kind == 2:
            seg = np.zeros(top, dtype=np.int64)
            seg[rng.integers(0, top)] = rng.integers(1, 2 * top)
        else:
            seg = rng.integers(0, 2, top)
        assert sliced(seg, top) == direct(seg, top), (seed, t, top)


def test_fig6_vertex_v5():
    # Fig. 6: v5's buckets {1: 2, 2: 2, 3: 1, 4: 0, 5: 0} give h = 2 with sum 3
    seg = np.array([2, 2, 1, 0, 0])
    assert direct(seg, 5) == (2, 3) == sliced(seg, 5)
