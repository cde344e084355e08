"""The seeded input generators: determinism, CSR well-formedness, RNG pin."""
import torch

import graphgen as gg


def test_splitmix64_published_vectors():
    # First outputs of SplitMix64 seeded with 1234567 and with 0, as listed
    # with the generator's reference implementation.
    x = gg.rand64(1234567, torch.arange(5))
    assert [int(v) & (2**64 - 1) for v in x.tolist()] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]
    assert int(gg.rand64(0, torch.arange(1))[0]) & (2**64 - 1) == 0xE220A8397B1DCDAF


def _check_csr(g):
    off = g.offsets.to(torch.int64)
    assert off[0].item() == 0 and off[-1].item() == g.m == g.cols.numel()
    assert bool((off[1:] >= off[:-1]).all())
    src, dst = g.edge_pairs()
    assert bool((dst >= 0).all()) and bool((dst < g.n).all())
    assert not bool((src == dst).any())
    key = src * g.n + dst
    assert bool((key[1:] > key[:-1]).all())          # sorted rows, no duplicates
    rev = torch.sort(dst * g.n + src).values
    assert torch.equal(rev, key)                     # symmetric


def test_generators_well_formed_and_deterministic():
    for make in (lambda: gg.er_gnp(2000, 8.0, 3), lambda: gg.er_gnm(5000, 12.0, 4),
                 lambda: gg.rmat(12, 16, 7), lambda: gg.rmat(12, 8, 7, n=3000),
                 lambda: gg.scaled_rmat_block(12, 2, 80, 0.6, 4)):
        a, b = make(), make()
        _check_csr(a)
        assert gg.fingerprint(a) == gg.fingerprint(b)
        assert torch.equal(a.cols, b.cols) and torch.equal(a.offsets, b.offsets)


def test_thread_count_independent():
    n0 = torch.get_num_threads()
    try:
        torch.set_num_threads(1)
        a = gg.rmat(11, 16, 5)
        torch.set_num_threads(max(2, n0))
        b = gg.rmat(11, 16, 5)
    finally:
        torch.set_num_threads(n0)
    assert gg.fingerprint(a) == gg.fingerprint(b)


def test_er10k_shape():
    g = gg.er_10k()
    _check_csr(g)
    assert g.n == 10_000
    assert 76_000 < g.m < 84_000          # E|m| = n * 8
    iso = int((g.degrees() == 0).sum())   # E = n e^-8 ~ 3.4
    assert iso <= 15


def test_planted_block_members_distinct():
    s, d, mem = gg.plant_block(1 << 16, 500, 0.6, 11)
    assert torch.unique(mem).numel() == 500
    frac = s.numel() / (500 * 499 / 2)
    assert 0.57 < frac < 0.63


def test_permutation_is_bijection():
    for bits in (1, 5, 16):
        x = torch.arange(1 << bits)
        assert torch.unique(gg.permute_pow2(x, bits, 9)).numel() == 1 << bits


def test_g1_shape():
    g = gg.g1()
    assert g.degrees().tolist() == [1, 1, 2, 3, 2, 5]
    assert g.m == 14


def test_pieces_below_the_32_bit_count_limit_give_the_same_csr():
    """CSR construction splits its inputs and key ranges into pieces; the
    result must not depend on the piece size."""
    ref = gg.rmat(12, 16, 3)
    old = gg._PIECE_MAX
    try:
        gg._PIECE_MAX = 3000
        small = gg.rmat(12, 16, 3)
    finally:
        gg._PIECE_MAX = old
    assert torch.equal(ref.offsets, small.offsets) and torch.equal(ref.cols, small.cols)


def test_mixed_batch_structure():
    b = gg.mixed_batch(24, 2, 5000, seed=31)
    assert b.num_graphs == 24 and b.vptr[0] == 0 and b.offsets[0] == 0
    assert int(b.offsets[-1]) == b.total_m
    for g in range(b.num_graphs):
        one = b.graph(g)
        _check_csr(one)
        assert one.n == int(b.vptr[g + 1] - b.vptr[g])
        if one.m:
            assert int(one.cols.max()) < one.n  # graph-local ids
    sizes = (b.vptr[1:] - b.vptr[:-1])
    assert int(sizes.min()) >= 2 and int(sizes.max()) <= 5000
    # deterministic
    assert torch.equal(gg.mixed_batch(24, 2, 5000, seed=31).cols, b.cols)


def test_lognormal_sizes_and_poisson_trace_statistics():
    s = gg.lognormal_sizes(20000, 20000, 1.5, 8_000_000, 2000).double()
    med = float(s.median())
    assert 18000 < med < 22000                       # median 20,000
    z = torch.log(s[(s > 2) & (s < 8_000_000)] / 20000)
    assert 1.4 < float(z.std()) < 1.6                # sigma 1.5
    t, pick = gg.poisson_trace(2000.0, 20.0, 2048, seed=2000)
    assert abs(t.numel() - 40000) < 4 * 200          # Poisson count, sd = 200
    gaps = torch.diff(t)
    assert (gaps > 0).all() and abs(float(gaps.mean()) - 1 / 2000) < 2e-5
    assert int(pick.min()) >= 0 and int(pick.max()) < 2048


def test_serving_pool_structure():
    p = gg.serving_pool(6, 500, 1.0, 4000, seed=9)
    assert p.num_graphs == 6
    for g in range(6):
        _check_csr(p.graph(g))
