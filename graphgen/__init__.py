"""Seeded synthetic graph inputs for the k-core decomposition path and its oracle.

This module builds graphs only: it holds none of the decomposition's arithmetic.
Both the HIP path (through the package's Python binding) and the CPU oracle read
the CSR arrays it produces, so parity never depends on how a graph was drawn.

Every random draw is the i-th output of a SplitMix64 stream (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
``z = seed + (i + 1) * 0x9E3779B97F4A7C15`` followed by the published
three-step finaliser.  It is evaluated with int64 tensor arithmetic (which wraps
modulo 2**64), so a graph is bit-identical on the CPU and on a GPU and for any
thread count.

Graph model (the paper's storage, Section II-B "Graph Storage"): an undirected
simple graph stored as CSR with both directions of every edge, rows sorted,
no self-loops and no duplicate entries.  ``m`` is the number of directed
entries, the |E| convention of the paper's dataset table (d_avg = |E|/|V|).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

__all__ = [
    "CSRGraph", "csr_from_pairs", "rand64", "uniform_u32", "stream_seed",
    "er_gnp", "er_gnm", "rmat", "plant_block", "permute_pow2",
    "g1", "complete", "cycle", "path", "star", "complete_bipartite",
    "hypercube", "circulant", "disjoint_union", "empty_graph", "from_edge_list",
    "er_10k", "rmat22", "rmat26_block", "fingerprint",
]

_MASK64 = (1 << 64) - 1


def _s64(x: int) -> int:
    """Reinterpret an unsigned 64-bit Python int as a signed int64 value."""
    x &= _MASK64
    return x - (1 << 64) if x >= (1 << 63) else x


_GOLD = _s64(0x9E3779B97F4A7C15)
_MIX1 = _s64(0xBF58476D1CE4E5B9)
_MIX2 = _s64(0x94D049BB133111EB)


def _lsr(x: torch.Tensor, s: int) -> torch.Tensor:
    """Logical right shift of int64 values (torch's >> is arithmetic)."""
    return (x >> s) & ((1 << (64 - s)) - 1)


def _mix(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _lsr(z, 30)) * _MIX1
    z = (z ^ _lsr(z, 27)) * _MIX2
    return z ^ _lsr(z, 31)


def _mix_int(z: int) -> int:
    z &= _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def stream_seed(*keys: int) -> int:
    """Derive an independent 64-bit stream seed from integer keys (host side)."""
    s = 0x5DEECE66D
    for k in keys:
        s = _mix_int(s + (int(k) + 1) * 0x9E3779B97F4A7C15)
    return _s64(s)


def rand64(seed: int, idx: torch.Tensor) -> torch.Tensor:
    """Output number ``idx`` of the SplitMix64 stream ``seed`` (int64 tensor)."""
    return _mix(seed + (idx + 1) * _GOLD)


def uniform_u32(seed: int, idx: torch.Tensor) -> torch.Tensor:
    """Uniform integers in [0, 2**32) from the top half of ``rand64``."""
    return _lsr(rand64(seed, idx), 32)


@dataclass
class CSRGraph:
    """An undirected simple graph in CSR form (both directions stored)."""

    name: str
    n: int
    m: int
    offsets: torch.Tensor  # int32 or int64, shape [n + 1]
    cols: torch.Tensor     # int32, shape [m]
    meta: dict = field(default_factory=dict)

    @property
    def offsets_i64(self) -> bool:
        return self.offsets.dtype == torch.int64

    def to(self, device) -> "CSRGraph":
        return CSRGraph(self.name, self.n, self.m, self.offsets.to(device),
                        self.cols.to(device), dict(self.meta))

    def with_offsets(self, dtype: torch.dtype) -> "CSRGraph":
        if dtype == torch.int32 and self.m >= 2**31:
            raise ValueError("int32 offsets cannot address m >= 2**31 entries")
        return CSRGraph(self.name, self.n, self.m, self.offsets.to(dtype),
                        self.cols, dict(self.meta))

    def degrees(self) -> torch.Tensor:
        o = self.offsets.to(torch.int64)
        return o[1:] - o[:-1]

    def edge_pairs(self):
        """(src, dst) int64 tensors of all directed entries."""
        deg = self.degrees()
        src = torch.repeat_interleave(torch.arange(self.n, device=deg.device), deg)
        return src, self.cols.to(torch.int64)


# torch.unique and boolean selection run on device libraries that index with
# 32-bit counts, so no single call may see 2**31 or more elements.
_PIECE_MAX = 1 << 30


def _unique_pieces(parts, lo: int, hi: int) -> list:
    """Sorted distinct values of the union of ``parts`` (all in [lo, hi)), as
    a list of ascending pieces covering consecutive value ranges."""
    total = sum(int(p.numel()) for p in parts)
    if total <= _PIECE_MAX or hi - lo <= 1:
        return [torch.unique(torch.cat(parts) if len(parts) > 1 else parts[0])]
    mid = lo + (hi - lo) // 2
    left = [p[p < mid] for p in parts]
    right = [p[p >= mid] for p in parts]
    del parts
    return _unique_pieces(left, lo, mid) + _unique_pieces(right, mid, hi)


def csr_from_pairs(n: int, src: torch.Tensor, dst: torch.Tensor, *,
                   offsets_dtype: torch.dtype = torch.int32, name: str = "graph",
                   meta: dict | None = None) -> CSRGraph:
    """Symmetrise, drop self-loops and duplicates, and sort into CSR."""
    parts = []
    for c0 in range(0, src.numel(), _PIECE_MAX):
        s = src[c0:c0 + _PIECE_MAX].to(torch.int64)
        d = dst[c0:c0 + _PIECE_MAX].to(torch.int64)
        keep = s != d
        s, d = s[keep], d[keep]
        parts += [s * n + d, d * n + s]
        del s, d, keep
    if not parts:
        parts = [torch.zeros(0, dtype=torch.int64, device=src.device)]
    # distinct keys, ascending: row-major CSR order
    pieces = _unique_pieces(parts, 0, max(n * n, 1))
    del parts
    counts = torch.zeros(n, dtype=torch.int64, device=pieces[0].device)
    cols = []
    for k in pieces:
        rows = torch.div(k, n, rounding_mode="floor")
        counts += torch.bincount(rows, minlength=n)
        cols.append((k - rows * n).to(torch.int32))
        del rows
    del pieces
    cols = torch.cat(cols) if len(cols) > 1 else cols[0]
    m = int(cols.numel())
    if offsets_dtype == torch.int32 and m >= 2**31:
        raise ValueError("graph too large for int32 offsets")
    offsets = torch.zeros(n + 1, dtype=torch.int64, device=cols.device)
    offsets[1:] = torch.cumsum(counts, 0)
    return CSRGraph(name, n, m, offsets.to(offsets_dtype), cols, meta or {})


def from_edge_list(n: int, edges, *, name: str = "graph",
                   offsets_dtype: torch.dtype = torch.int32) -> CSRGraph:
    """CSR of an explicit undirected edge list [(u, v), ...]."""
    if len(edges) == 0:
        src = torch.zeros(0, dtype=torch.int64)
        dst = torch.zeros(0, dtype=torch.int64)
    else:
        t = torch.tensor(edges, dtype=torch.int64)
        src, dst = t[:, 0], t[:, 1]
    return csr_from_pairs(n, src, dst, offsets_dtype=offsets_dtype, name=name)


# ---------------------------------------------------------------------------
# Small structured graphs (worked example and closed-form families)
# ---------------------------------------------------------------------------

def g1() -> CSRGraph:
    """The paper's running example G1 (Fig. 1), with the edge list implied by
    the text: v5 has degree 5 (its h-index starts at 5, Section II-C), v5's
    neighbours hold degrees 1,1,2,2,3 (Fig. 6), and v3 and v5 are the two
    vertices whose residual degree falls under their coreness (Section III-A).
    """
    edges = [(0, 5), (1, 5), (2, 5), (3, 5), (4, 5), (2, 3), (3, 4)]
    return from_edge_list(6, edges, name="G1")


def empty_graph(n: int) -> CSRGraph:
    return from_edge_list(n, [], name=f"empty{n}")


def complete(n: int) -> CSRGraph:
    return from_edge_list(n, [(i, j) for i in range(n) for j in range(i + 1, n)],
                          name=f"K{n}")


def cycle(n: int) -> CSRGraph:
    return from_edge_list(n, [(i, (i + 1) % n) for i in range(n)], name=f"C{n}")


def path(n: int) -> CSRGraph:
    i = torch.arange(max(n - 1, 0), dtype=torch.int64)
    return csr_from_pairs(n, i, i + 1, name=f"P{n}")


def star(leaves: int) -> CSRGraph:
    i = torch.arange(1, leaves + 1, dtype=torch.int64)
    return csr_from_pairs(leaves + 1, torch.zeros_like(i), i, name=f"star{leaves}")


def complete_bipartite(a: int, b: int) -> CSRGraph:
    u = torch.arange(a, dtype=torch.int64).repeat_interleave(b)
    v = a + torch.arange(b, dtype=torch.int64).repeat(a)
    return csr_from_pairs(a + b, u, v, name=f"K{a},{b}")


def hypercube(d: int) -> CSRGraph:
    n = 1 << d
    v = torch.arange(n, dtype=torch.int64)
    src = torch.cat([v for _ in range(d)]) if d else v[:0]
    dst = torch.cat([v ^ (1 << b) for b in range(d)]) if d else v[:0]
    return csr_from_pairs(n, src, dst, name=f"Q{d}")


def circulant(n: int, jumps) -> CSRGraph:
    v = torch.arange(n, dtype=torch.int64)
    src = torch.cat([v for _ in jumps])
    dst = torch.cat([(v + j) % n for j in jumps])
    return csr_from_pairs(n, src, dst, name=f"circ{n}{list(jumps)}")


def disjoint_union(*graphs: CSRGraph) -> CSRGraph:
    srcs, dsts, base = [], [], 0
    for g in graphs:
        s, d = g.edge_pairs()
        srcs.append(s + base)
        dsts.append(d + base)
        base += g.n
    return csr_from_pairs(base, torch.cat(srcs), torch.cat(dsts),
                          name="+".join(g.name for g in graphs))


# ---------------------------------------------------------------------------
# Random graph models
# ---------------------------------------------------------------------------

def er_gnp(n: int, avg_deg: float, seed: int, *, device="cpu",
           offsets_dtype=torch.int32, row_chunk: int = 512) -> CSRGraph:
    """Exact Erdos-Renyi G(n, p) with p = avg_deg / (n - 1): every pair i < j
    is kept iff its 32-bit draw is below round(p * 2**32).  O(n**2) draws, so
    meant for n up to a few tens of thousands."""
    p = avg_deg / max(n - 1, 1)
    thresh = int(round(p * 2**32))
    s = stream_seed(seed, 0xE5)
    srcs, dsts = [], []
    j = torch.arange(n, dtype=torch.int64, device=device)
    for i0 in range(0, n, row_chunk):
        i = torch.arange(i0, min(n, i0 + row_chunk), dtype=torch.int64, device=device)
        idx = i[:, None] * n + j[None, :]
        keep = (j[None, :] > i[:, None]) & (uniform_u32(s, idx) < thresh)
        ii, jj = torch.nonzero(keep, as_tuple=True)
        srcs.append(i[ii])
        dsts.append(jj)
    return csr_from_pairs(n, torch.cat(srcs), torch.cat(dsts), offsets_dtype=offsets_dtype,
                          name=f"ER-gnp(n={n},d={avg_deg},seed={seed})",
                          meta={"model": "gnp", "p_u32": thresh, "seed": seed})


def er_gnm(n: int, avg_deg: float, seed: int, *, device="cpu",
           offsets_dtype=torch.int32) -> CSRGraph:
    """Erdos-Renyi by M = round(avg_deg * n / 2) uniform endpoint pairs drawn
    with replacement; self-loops and repeats are then dropped (a G(n, M)
    approximation of G(n, p) for sizes where O(n**2) draws are too many)."""
    M = int(round(avg_deg * n / 2))
    s = stream_seed(seed, 0xE6)
    e = torch.arange(M, dtype=torch.int64, device=device)
    src = _lsr(rand64(s, 2 * e), 1) % n
    dst = _lsr(rand64(s, 2 * e + 1), 1) % n
    return csr_from_pairs(n, src, dst, offsets_dtype=offsets_dtype,
                          name=f"ER-gnm(n={n},d={avg_deg},seed={seed})",
                          meta={"model": "gnm", "M": M, "seed": seed})


def permute_pow2(x: torch.Tensor, bits: int, seed: int) -> torch.Tensor:
    """A seeded bijection of [0, 2**bits): three rounds of (multiply by an odd
    constant, xorshift, add) modulo 2**bits; each step is invertible."""
    if bits == 0:
        return x
    mask = (1 << bits) - 1
    sh = (bits + 1) // 2
    for r in range(3):
        odd = (stream_seed(seed, r, 1) | 1) & mask | 1
        add = stream_seed(seed, r, 2) & mask
        x = (x * odd) & mask
        x = x ^ (x >> sh)
        x = (x + add) & mask
    return x


def _permute_n(x: torch.Tensor, n: int, seed: int) -> torch.Tensor:
    """Bijection of [0, n) by cycle-walking ``permute_pow2`` on the next power of 2."""
    bits = max(1, (n - 1).bit_length())
    y = permute_pow2(x, bits, seed)
    for _ in range(1 << 12):
        bad = y >= n
        if not bool(bad.any()):
            return y
        y = torch.where(bad, permute_pow2(y, bits, seed), y)
    raise RuntimeError("cycle walk did not converge")


def _rmat_endpoints(e: torch.Tensor, scale: int, seed: int, thr) -> tuple:
    """Graph500-style recursive quadrant descent for edge ids ``e`` (no noise)."""
    A, AB, ABC = thr
    src = torch.zeros_like(e)
    dst = torch.zeros_like(e)
    h = None
    for lvl in range(scale):
        if lvl % 2 == 0:
            h = rand64(seed, e * 32 + lvl // 2)
            r = _lsr(h, 32)
        else:
            r = h & 0xFFFFFFFF
        q = (r >= A).to(torch.int64) + (r >= AB).to(torch.int64) + (r >= ABC).to(torch.int64)
        src = (src << 1) | (q >> 1)
        dst = (dst << 1) | (q & 1)
    return src, dst


def rmat(scale: int, edge_factor: int, seed: int, *, a=0.57, b=0.19, c=0.19,
         n: int | None = None, permute: bool = True, device="cpu",
         offsets_dtype=torch.int32, chunk: int = 1 << 25,
         extra_pairs=None, name: str | None = None) -> CSRGraph:
    """R-MAT graph: ``edge_factor * n`` generated edges over n = 2**scale
    vertices (or a given n <= 2**scale, endpoints >= n redrawn), quadrant
    probabilities (a, b, c, 1-a-b-c) quantised to 1/2**32, then a seeded
    vertex relabelling, symmetrisation, dedup and self-loop removal.
    ``extra_pairs`` (src, dst) are appended before the CSR is built."""
    if n is None:
        n = 1 << scale
    assert n <= (1 << scale)
    thr = (int(round(a * 2**32)), int(round((a + b) * 2**32)), int(round((a + b + c) * 2**32)))
    M = edge_factor * n
    s = stream_seed(seed, 0x4D)
    psd = stream_seed(seed, 0x50)
    srcs, dsts = [], []
    for e0 in range(0, M, chunk):
        e = torch.arange(e0, min(M, e0 + chunk), dtype=torch.int64, device=device)
        src, dst = _rmat_endpoints(e, scale, s, thr)
        for attempt in range(1, 257):
            bad = (src >= n) | (dst >= n)
            if not bool(bad.any()):
                break
            rs, rd = _rmat_endpoints(e[bad] + attempt * (1 << 40), scale, s, thr)
            src[bad], dst[bad] = rs, rd
        else:
            keep = (src < n) & (dst < n)
            src, dst = src[keep], dst[keep]
        if permute:
            src = _permute_n(src, n, psd)
            dst = _permute_n(dst, n, psd)
        srcs.append(src)
        dsts.append(dst)
    if extra_pairs is not None:
        srcs.append(extra_pairs[0].to(device))
        dsts.append(extra_pairs[1].to(device))
    src = torch.cat(srcs)
    dst = torch.cat(dsts)
    del srcs, dsts
    return csr_from_pairs(n, src, dst, offsets_dtype=offsets_dtype,
                          name=name or f"RMAT(scale={scale},ef={edge_factor},seed={seed})",
                          meta={"model": "rmat", "scale": scale, "edge_factor": edge_factor,
                                "abc": (a, b, c), "seed": seed})


def plant_block(n: int, size: int, p: float, seed: int, *, device="cpu"):
    """Pairs of a planted dense block: ``size`` distinct vertices of [0, n)
    (a seeded bijection's images of 0..size-1), each of their pairs kept with
    probability p.  Returns (src, dst, members)."""
    members = _permute_n(torch.arange(size, dtype=torch.int64, device=device), n,
                         stream_seed(seed, 0xB1))
    thresh = int(round(p * 2**32))
    s = stream_seed(seed, 0xB2)
    i = torch.arange(size, dtype=torch.int64, device=device)
    idx = i[:, None] * size + i[None, :]
    keep = (i[None, :] > i[:, None]) & (uniform_u32(s, idx) < thresh)
    ii, jj = torch.nonzero(keep, as_tuple=True)
    return members[ii], members[jj], members


def edit_edges(g: CSRGraph, delete_frac: float, insert: int, seed: int) -> tuple:
    """A changed copy of g for core maintenance: each undirected edge is
    deleted with probability `delete_frac` (its 32-bit draw below
    delete_frac * 2**32), then `insert` random vertex pairs are added (pairs
    that are loops or already edges add nothing).  Returns (new graph, number
    of undirected edges actually inserted), offsets of g's dtype."""
    src, dst = g.edge_pairs()
    upper = src < dst  # one entry per undirected edge
    s, d = src[upper], dst[upper]
    key = s * g.n + d
    draw = uniform_u32(stream_seed(seed, 0xDE1), key)
    keep = draw >= int(round(delete_frac * 2**32))
    s, d = s[keep], d[keep]
    ins = 0
    if insert > 0 and g.n > 1:
        idx = torch.arange(insert, device=src.device)
        a = (uniform_u32(stream_seed(seed, 0x1A5), idx) % g.n).to(torch.int64)
        b = (uniform_u32(stream_seed(seed, 0x1A6), idx) % g.n).to(torch.int64)
        lo, hi = torch.minimum(a, b), torch.maximum(a, b)
        new = torch.unique(lo * g.n + hi)
        new = new[(new // g.n) != (new % g.n)]
        old = torch.unique(s * g.n + d)
        fresh = new[~torch.isin(new, old)]
        ins = int(fresh.numel())
        s = torch.cat([s, fresh // g.n])
        d = torch.cat([d, fresh % g.n])
    h = csr_from_pairs(g.n, s, d, offsets_dtype=g.offsets.dtype,
                       name=f"{g.name}+edit(del={delete_frac},ins={insert},seed={seed})")
    return h, ins


def fingerprint(g: CSRGraph) -> str:
    """A 64-bit checksum of the CSR (n, m and every (row, col) entry)."""
    src, dst = g.edge_pairs()
    h = rand64(0x1234567, src * 4294967296 + dst)
    acc = int(h.sum().item()) & _MASK64 if g.m else 0
    acc = _mix_int(acc ^ _mix_int(g.n) ^ (_mix_int(g.m) << 1))
    return f"{g.n}:{g.m}:{acc:016x}"


# ---------------------------------------------------------------------------
# The named workloads
# ---------------------------------------------------------------------------

def er_10k(seed: int = 1, device="cpu") -> CSRGraph:
    """G(n=10,000, avg degree 8), int32 CSR."""
    g = er_gnp(10_000, 8.0, seed, device=device)
    g.name = f"ER-10k(seed={seed})"
    return g


def rmat22(seed: int = 22, device="cpu") -> CSRGraph:
    """R-MAT scale 22, edge factor 16, (0.57, 0.19, 0.19, 0.05), permuted, int32."""
    return rmat(22, 16, seed, device=device, offsets_dtype=torch.int32,
                name=f"RMAT-22(ef=16,seed={seed})")


def rmat26_block(seed: int = 26, block_seed: int = 2601, device="cpu",
                 block: int = 3000, p: float = 0.6) -> CSRGraph:
    """R-MAT scale 26, edge factor 16, plus a planted block of 3,000 vertices
    at pair probability 0.6; int64 offsets, int32 cols."""
    n = 1 << 26
    bs, bd, _ = plant_block(n, block, p, block_seed, device=device)
    g = rmat(26, 16, seed, device=device, offsets_dtype=torch.int64,
             extra_pairs=(bs, bd), name=f"RMAT-26+block(seed={seed},block_seed={block_seed})")
    g.meta.update({"block": block, "block_p": p, "block_seed": block_seed})
    return g


def scaled_rmat_block(scale: int, seed: int, block: int, p: float, block_seed: int,
                      device="cpu", offsets_dtype=torch.int32) -> CSRGraph:
    """Smaller relative of the RMAT-26 + block workload (same recipe, smaller
    scale and block), for parity tests the oracle finishes in seconds."""
    n = 1 << scale
    bs, bd, _ = plant_block(n, block, p, block_seed, device=device)
    return rmat(scale, 16, seed, device=device, offsets_dtype=offsets_dtype,
                extra_pairs=(bs, bd),
                name=f"RMAT-{scale}+block{block}(seed={seed})")


def log_uniform_int(seed: int, idx: torch.Tensor, lo: int, hi: int) -> torch.Tensor:
    """Integers log-uniform on [lo, hi] (exp of a 32-bit uniform, float64)."""
    u = uniform_u32(seed, idx).to(torch.float64) / 2**32
    return torch.floor(torch.exp(math.log(lo) + u * (math.log(hi + 1) - math.log(lo)))).to(torch.int64).clamp(lo, hi)


# ---------------------------------------------------------------------------
# Batches of independent graphs (packed multi-CSR)
# ---------------------------------------------------------------------------

@dataclass
class GraphBatch:
    """Many graphs in one packed CSR: graph g owns global vertices
    [vptr[g], vptr[g+1]); offsets are global int64 positions into cols; cols
    hold graph-local neighbour ids."""

    name: str
    vptr: torch.Tensor     # int64 [G + 1]
    offsets: torch.Tensor  # int64 [total_n + 1]
    cols: torch.Tensor     # int32 [total_m]
    meta: dict = field(default_factory=dict)

    @property
    def num_graphs(self) -> int:
        return self.vptr.numel() - 1

    @property
    def total_n(self) -> int:
        return int(self.vptr[-1])

    @property
    def total_m(self) -> int:
        return int(self.cols.numel())

    def to(self, device) -> "GraphBatch":
        return GraphBatch(self.name, self.vptr.to(device), self.offsets.to(device),
                          self.cols.to(device), dict(self.meta))

    def graph(self, g: int) -> CSRGraph:
        """Graph g on its own, with int32 or int64 offsets as it needs."""
        x0, x1 = int(self.vptr[g]), int(self.vptr[g + 1])
        off = self.offsets[x0:x1 + 1].to(torch.int64)
        e0 = int(off[0])
        off = off - e0
        m = int(off[-1])
        cols = self.cols[e0:e0 + m]
        dt = torch.int32 if m < 2**31 else torch.int64
        return CSRGraph(f"{self.name}[{g}]", x1 - x0, m, off.to(dt), cols, {})


def pack_pairs(sizes: torch.Tensor, gsrc: torch.Tensor, gdst: torch.Tensor, name: str,
               meta: dict | None = None) -> GraphBatch:
    """Packed multi-CSR of disjoint graphs from global endpoint pairs (graph g's
    local vertex v is global id vptr[g] + v): symmetrised, deduplicated,
    self-loops removed."""
    sizes = sizes.to(torch.int64)
    vptr = torch.zeros(sizes.numel() + 1, dtype=torch.int64, device=sizes.device)
    vptr[1:] = torch.cumsum(sizes, 0)
    total = int(vptr[-1])
    g = csr_from_pairs(total, gsrc, gdst, offsets_dtype=torch.int64, name=name)
    # global -> graph-local column ids, in pieces of the position range
    dv = g.cols.device
    vp = vptr.to(dv)
    cols = g.cols
    for c0 in range(0, g.m, _PIECE_MAX):
        c1 = min(g.m, c0 + _PIECE_MAX)
        pos = torch.arange(c0, c1, device=dv)
        row = torch.searchsorted(g.offsets, pos, right=True) - 1
        graph = torch.searchsorted(vp, row, right=True) - 1
        cols[c0:c1] -= vp[graph].to(torch.int32)
        del pos, row, graph
    return GraphBatch(name, vp, g.offsets, cols, meta or {})


def batch_sizes(count: int, lo: int, hi: int, seed: int) -> torch.Tensor:
    """Vertex counts log-uniform on [lo, hi] (computed on the CPU, so identical
    on every device)."""
    return log_uniform_int(stream_seed(seed, 0x51), torch.arange(count), lo, hi)


_RMAT_THR = (int(round(0.57 * 2**32)), int(round(0.76 * 2**32)), int(round(0.95 * 2**32)))


def _rmat_local_pairs(n: int, ef: int, gs: int, device):
    """ef * n R-MAT endpoint pairs over [0, n) (scale ceil(log2 n), endpoints
    >= n redrawn, (0.57, 0.19, 0.19)), relabelled by a seeded bijection."""
    scale = max(1, (n - 1).bit_length())
    e = torch.arange(ef * n, dtype=torch.int64, device=device)
    s, t = _rmat_endpoints(e, scale, gs, _RMAT_THR)
    for attempt in range(1, 257):
        bad = (s >= n) | (t >= n)
        if not bool(bad.any()):
            break
        rs, rd = _rmat_endpoints(e[bad] + attempt * (1 << 40), scale, gs, _RMAT_THR)
        s[bad], t[bad] = rs, rd
    keep = (s < n) & (t < n)
    s, t = s[keep], t[keep]
    p = stream_seed(gs, 0x50)
    return _permute_n(s, n, p), _permute_n(t, n, p)


def mixed_batch(count: int = 4096, lo: int = 200, hi: int = 200_000, seed: int = 4096,
                device="cpu", progress=None) -> GraphBatch:
    """The batched workload: `count` graphs with vertex counts log-uniform on
    [lo, hi]; even-indexed graphs Erdos-Renyi G(n, M) with average degree
    uniform on [4, 32], odd-indexed R-MAT (scale ceil(log2 n), endpoints >= n
    redrawn) with edge factor uniform on [8, 16] and (0.57, 0.19, 0.19).
    Graph g draws from streams seeded by (seed, g).  `progress(g)`, if
    given, is called every 256 graphs."""
    sizes = batch_sizes(count, lo, hi, seed)
    u = uniform_u32(stream_seed(seed, 0x52), torch.arange(count)).to(torch.float64) / 2**32
    srcs, dsts = [], []
    vbase = 0
    for g in range(count):
        if progress is not None and g % 256 == 0:
            progress(g)
        n = int(sizes[g])
        gs = stream_seed(seed, g)
        if g % 2 == 0:
            d = 4.0 + 28.0 * float(u[g])
            M = int(round(d * n / 2))
            e = torch.arange(M, dtype=torch.int64, device=device)
            s = _lsr(rand64(gs, 2 * e), 1) % n
            t = _lsr(rand64(gs, 2 * e + 1), 1) % n
        else:
            ef = min(8 + int(float(u[g]) * 9), 16)
            s, t = _rmat_local_pairs(n, ef, gs, device)
        srcs.append(s + vbase)
        dsts.append(t + vbase)
        vbase += n
    return pack_pairs(sizes.to(device), torch.cat(srcs), torch.cat(dsts),
                      name=f"batch(count={count},n=[{lo},{hi}],seed={seed})",
                      meta={"count": count, "lo": lo, "hi": hi, "seed": seed})


# ---------------------------------------------------------------------------
# Serving workload: a pool of request graphs and a Poisson arrival trace
# ---------------------------------------------------------------------------

def std_normal(seed: int, idx: torch.Tensor) -> torch.Tensor:
    """Standard normal deviates (Box-Muller on two counter-based uniforms)."""
    u1 = (uniform_u32(seed, 2 * idx).to(torch.float64) + 0.5) / 2**32
    u2 = (uniform_u32(seed, 2 * idx + 1).to(torch.float64) + 0.5) / 2**32
    return torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)


def lognormal_sizes(count: int, median: int, sigma: float, cap: int, seed: int,
                    lo: int = 2) -> torch.Tensor:
    """Vertex counts floor(median * exp(sigma * z)), clamped to [lo, cap]."""
    z = std_normal(stream_seed(seed, 0x4C), torch.arange(count))
    return torch.floor(median * torch.exp(sigma * z)).to(torch.int64).clamp(lo, cap)


def serving_pool(count: int = 2048, median: int = 20_000, sigma: float = 1.5, cap: int = 8_000_000,
                 edge_factor: int = 16, seed: int = 2000, device="cpu", progress=None) -> GraphBatch:
    """The pool the serving trace draws from: `count` R-MAT graphs (edge factor
    16, (0.57, 0.19, 0.19)) with lognormal vertex counts (median 20,000,
    sigma 1.5, capped at 8,000,000), packed like a batch."""
    sizes = lognormal_sizes(count, median, sigma, cap, seed)
    srcs, dsts, vbase = [], [], 0
    for g in range(count):
        if progress is not None and g % 256 == 0:
            progress(g)
        n = int(sizes[g])
        s, t = _rmat_local_pairs(n, edge_factor, stream_seed(seed, 0x10000 + g), device)
        srcs.append(s + vbase)
        dsts.append(t + vbase)
        vbase += n
    return pack_pairs(sizes.to(device), torch.cat(srcs), torch.cat(dsts),
                      name=f"serving-pool(count={count},median={median},sigma={sigma},seed={seed})",
                      meta={"count": count, "median": median, "sigma": sigma, "cap": cap,
                            "edge_factor": edge_factor, "seed": seed})


def poisson_trace(rate: float, duration: float, pool_size: int, seed: int = 2000):
    """Arrival times (seconds, float64, increasing) of a Poisson stream at
    `rate` per second over `duration` seconds, and the pool graph each
    request asks for (uniform over the pool).  CPU tensors."""
    est = int(rate * duration * 1.2 + 64)
    u = (uniform_u32(stream_seed(seed, 0x41), torch.arange(est)).to(torch.float64) + 0.5) / 2**32
    t = torch.cumsum(-torch.log(u) / rate, 0)
    t = t[t < duration]
    pick = uniform_u32(stream_seed(seed, 0x42), torch.arange(t.numel())) % pool_size
    return t, pick.to(torch.int64)
