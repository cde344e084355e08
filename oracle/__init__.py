"""CPU oracle for k-core decomposition -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The GPU library neither imports nor links any of
it, and it imports nothing from the GPU library: the two share no code.

Routines (each cites the passage of the paper it follows):

* ``bz_coreness``    -- Batagelj-Zaversnik bucket peel (C, O(n + m)); the
  plain definition of coreness from Section I.  Related work, Section VI-A.
* ``hindex_jacobi``  -- the Index2core paradigm (Section II-A, Alg. 2) in
  synchronous rounds, h-index by sorting (C).
* ``index2core``     -- CntCore (Section IV-A, Alg. 5) and NbrCore (the
  Index2core baseline of Section V) in synchronous rounds, with work counts
  (C).
* ``peel_gpp``       -- General Parallel Peel (Section II-C, Alg. 3; the GPP
  baseline of Section V), serially, with its iteration count (C).
* ``peel_static``    -- PeelOne without the dynamic frontier (the variant of
  Table IV), serially, with its iteration count (C).
* ``hindex_jacobi_from`` -- the same iteration started from upper bounds of
  the coreness (core maintenance after edge changes), never raising a value
  (C).
* ``brute_coreness`` -- the definition literally: for each k, delete vertices
  of degree < k until none is left; survivors form the k-core (pure Python,
  tiny graphs only).
* ``peelone_trace``  -- PeelOne (Section III-C, Alg. 4) executed serially:
  levels k = 1, 2, ...; frontier = residual vertices whose value equals k;
  the assertion decrement of Section III-B on neighbours valued above k; a
  neighbour whose decrement lands on k joins the level's dynamic frontier.
  Records per-level frontier sets and value trajectories (pure Python).
* ``histocore_trace`` -- HistoCore (Section IV-B, Alg. 6) executed serially
  in separate SumHisto / UpdateHisto phases (pure Python): InitHisto over
  neighbour values min(core[u], core[v]), the cnt-based frontier of Theorem 2,
  the reverse summation of Step II, and the N1/N3 histogram updates of
  Section IV-B-1 with exact crossing detection.

Readings of points where the paper is silent or garbled (all listed in the
design notes):
  * a vertex of degree 0 has coreness 0 (definition, Section I);
  * the assertion decrement returns the value it read, and a vertex joins the
    dynamic frontier iff that value was k + 1 (once per vertex);
  * SumHisto sums buckets from the old value downwards and stops at the first
    k whose running sum reaches k (so Fig. 6 yields h(v5) = 2 with sum 3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from collections import deque

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into oracle/_liboracle.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC],
                       check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_bz.restype = ctypes.c_int
        lib.oracle_bz.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p]
        lib.oracle_hindex_jacobi.restype = ctypes.c_int64
        lib.oracle_hindex_jacobi.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]
        lib.oracle_index2core.restype = ctypes.c_int
        lib.oracle_index2core.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_peel_gpp.restype = ctypes.c_int64
        lib.oracle_peel_gpp.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]
        lib.oracle_peel_static.restype = ctypes.c_int64
        lib.oracle_peel_static.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p]
        lib.oracle_hindex_jacobi_from.restype = ctypes.c_int64
        lib.oracle_hindex_jacobi_from.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def _csr_np(offsets, cols):
    """CSR as contiguous numpy (int64 offsets, int32 cols) from numpy or torch."""
    if hasattr(offsets, "cpu"):
        offsets = offsets.cpu().numpy()
    if hasattr(cols, "cpu"):
        cols = cols.cpu().numpy()
    off = np.ascontiguousarray(np.asarray(offsets), dtype=np.int64)
    adj = np.ascontiguousarray(np.asarray(cols), dtype=np.int32)
    return off, adj


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def bz_coreness(offsets, cols) -> np.ndarray:
    """Coreness of every vertex (int32[n]) by the Batagelj-Zaversnik peel."""
    off, adj = _csr_np(offsets, cols)
    n = off.shape[0] - 1
    core = np.zeros(max(n, 0), dtype=np.int32)
    rc = _load().oracle_bz(n, _ptr(off), _ptr(adj) if adj.size else None, _ptr(core))
    if rc != 0:
        raise RuntimeError(f"oracle_bz failed with {rc}")
    return core


def hindex_jacobi(offsets, cols, max_rounds: int = 1 << 30):
    """Synchronous h-index iteration from the degrees.

    Returns (x, changed_per_round, changed_round_of): values after the last
    round run, the number of changed vertices in each round that changed
    something, and for each vertex the last round that changed it (0 = never).
    """
    off, adj = _csr_np(offsets, cols)
    n = off.shape[0] - 1
    x = np.zeros(max(n, 0), dtype=np.int32)
    cap = int(min(max_rounds, max(n, 1) + 1))
    per_round = np.zeros(cap, dtype=np.int64)
    last = np.zeros(max(n, 0), dtype=np.int32)
    r = _load().oracle_hindex_jacobi(n, _ptr(off), _ptr(adj) if adj.size else None, cap,
                                     _ptr(x), _ptr(per_round), _ptr(last))
    if r < 0:
        raise RuntimeError(f"oracle_hindex_jacobi failed with {r}")
    return x, per_round[:r].tolist(), last


INDEX2CORE_COUNTS = ("rounds_changed", "rounds_run", "active", "hindex_computed", "edges_cnt",
                     "edges_hindex", "edges_mark", "activations")


def index2core(offsets, cols, variant: str):
    """CntCore (Alg. 5) or NbrCore in synchronous rounds from the degrees,
    every h-index recomputed from the neighbours' values (no maintained
    histogram).  Returns (coreness, {count name: value}) with the counts of
    INDEX2CORE_COUNTS."""
    mode = {"nbrcore": 0, "cntcore": 1}[variant]
    off, adj = _csr_np(offsets, cols)
    n = off.shape[0] - 1
    x = np.zeros(max(n, 0), dtype=np.int32)
    out = np.zeros(8, dtype=np.int64)
    r = _load().oracle_index2core(n, _ptr(off), _ptr(adj) if adj.size else None, mode, _ptr(x), _ptr(out))
    if r < 0:
        raise RuntimeError(f"oracle_index2core failed with {r}")
    return x, dict(zip(INDEX2CORE_COUNTS, (int(v) for v in out)))


def peel_gpp(offsets, cols):
    """General Parallel Peel (Alg. 3, Section II-C), serially: returns
    (coreness, iterations, decrements).  k starts at 0 with every vertex
    residual; each while-loop iteration raises k by one when no residual
    vertex has degree <= k, then scans (possibly finding nobody) and
    scatters.  One decrement per edge from a removed vertex to a residual
    one."""
    off, adj = _csr_np(offsets, cols)
    n = off.shape[0] - 1
    x = np.zeros(max(n, 0), dtype=np.int32)
    dec = np.zeros(1, dtype=np.int64)
    r = _load().oracle_peel_gpp(n, _ptr(off), _ptr(adj) if adj.size else None, _ptr(x), _ptr(dec))
    if r < 0:
        raise RuntimeError(f"oracle_peel_gpp failed with {r}")
    return x, int(r), int(dec[0])


def peel_static(offsets, cols):
    """PeelOne without the dynamic frontier (Table IV's variant), serially:
    returns (coreness, iterations), iterations counting every scan that found
    a vertex at the current level (sub-iterations included)."""
    off, adj = _csr_np(offsets, cols)
    n = off.shape[0] - 1
    x = np.zeros(max(n, 0), dtype=np.int32)
    r = _load().oracle_peel_static(n, _ptr(off), _ptr(adj) if adj.size else None, _ptr(x))
    if r < 0:
        raise RuntimeError(f"oracle_peel_static failed with {r}")
    return x, int(r)


def hindex_jacobi_from(offsets, cols, x0, add: int = 0, max_rounds: int = 1 << 30):
    """The synchronous h-index iteration started from upper bounds x0 (+ add)
    of the coreness, capped by the degree, each round keeping the smaller of a
    vertex's value and the h-index of its neighbours' values (core
    maintenance on a changed graph).  Returns as ``hindex_jacobi``."""
    off, adj = _csr_np(offsets, cols)
    n = off.shape[0] - 1
    start = np.ascontiguousarray(np.asarray(x0, dtype=np.int32))
    if start.shape != (max(n, 0),):
        raise ValueError("x0 must hold one value per vertex")
    x = np.zeros(max(n, 0), dtype=np.int32)
    cap = int(min(max_rounds, max(n, 1) + 1))
    per_round = np.zeros(cap, dtype=np.int64)
    last = np.zeros(max(n, 0), dtype=np.int32)
    r = _load().oracle_hindex_jacobi_from(n, _ptr(off), _ptr(adj) if adj.size else None, _ptr(start),
                                          int(add), cap, _ptr(x), _ptr(per_round), _ptr(last))
    if r < 0:
        raise RuntimeError(f"oracle_hindex_jacobi_from failed with {r}")
    return x, per_round[:r].tolist(), last


def _adjacency(offsets, cols):
    off, adj = _csr_np(offsets, cols)
    n = off.shape[0] - 1
    return n, [adj[off[v]:off[v + 1]].tolist() for v in range(n)]


def brute_coreness(n: int, edges) -> list:
    """The definition of Section I, literally, for tiny graphs: the k-core is
    what remains after repeatedly deleting any vertex with fewer than k
    neighbours left; core(v) is the largest k whose k-core contains v."""
    nbr = [set() for _ in range(n)]
    for u, v in edges:
        if u != v:
            nbr[u].add(v)
            nbr[v].add(u)
    core = [0] * n
    k = 1
    while True:
        alive = set(range(n))
        shrinking = True
        while shrinking:
            shrinking = False
            for v in sorted(alive):
                if len(nbr[v] & alive) < k:
                    alive.discard(v)
                    shrinking = True
        if not alive:
            return core
        for v in alive:
            core[v] = k
        k += 1


def peelone_trace(offsets, cols) -> dict:
    """PeelOne (Alg. 4) run serially; see the module docstring.

    Returns dict with ``core`` (list), ``levels`` (list of dicts with k,
    ``scan`` = frontier found by the scan, ``dynamic`` = vertices asserted into
    the level's queue, in order), and ``trajectory`` (per vertex, the list of
    values it took, starting at its degree).
    """
    n, nbr = _adjacency(offsets, cols)
    core = [len(nbr[v]) for v in range(n)]
    trajectory = [[core[v]] for v in range(n)]
    residual = {v for v in range(n) if core[v] > 0}
    out = [0] * n
    levels = []
    k = 0
    while residual:
        k += 1
        scan = sorted(v for v in residual if core[v] == k)
        queue = deque(scan)
        dynamic = []
        while queue:
            v = queue.popleft()
            residual.discard(v)
            out[v] = k
            for u in nbr[v]:
                if core[u] > k:
                    old = core[u]
                    core[u] = old - 1 if old > k else k  # the assertion decrement
                    trajectory[u].append(core[u])
                    if old == k + 1:
                        queue.append(u)
                        dynamic.append(u)
        levels.append({"k": k, "scan": scan, "dynamic": dynamic})
    return {"core": out, "levels": levels, "trajectory": trajectory}


def histocore_trace(offsets, cols) -> dict:
    """HistoCore (Alg. 6) run serially with separate phases; see the module
    docstring.  Returns dict with ``core``, ``init_histo`` (per vertex, list
    indexed 0..deg(v) with bucket 0 unused), ``frontiers`` (V_cnt of each
    iteration, sorted), ``iterations`` (l2) and ``cnt_ok`` (whether
    histo[v][core[v]] equalled the number of neighbours valued >= core[v] for
    every vertex after every iteration).
    """
    n, nbr = _adjacency(offsets, cols)
    core = [len(nbr[v]) for v in range(n)]
    oldcore = [0] * n
    histo = [[0] * (len(nbr[v]) + 1) for v in range(n)]
    for v in range(n):  # InitHisto
        for u in nbr[v]:
            histo[v][min(core[u], core[v])] += 1
    init_histo = [list(h) for h in histo]
    vcnt = [v for v in range(n) if core[v] > 0 and histo[v][core[v]] < core[v]]
    frontiers = []
    cnt_ok = True
    while vcnt:
        frontiers.append(sorted(vcnt))
        changed = []
        for v in vcnt:  # SumHisto
            core_old = core[v]
            s = 0
            k = core_old
            while True:
                s += histo[v][k]
                if s >= k:
                    break
                k -= 1
            if k != core_old:
                core[v] = k
                oldcore[v] = core_old
                histo[v][k] = s
                changed.append(v)
        nxt = []
        for v in changed:  # UpdateHisto
            for u in nbr[v]:
                if core[u] > core[v]:
                    b = min(oldcore[v], core[u])
                    c = histo[u][b]
                    histo[u][b] -= 1
                    histo[u][core[v]] += 1
                    if oldcore[v] >= core[u] and c == core[u]:
                        nxt.append(u)
        vcnt = nxt
        for v in range(n):
            if core[v] > 0:
                want = sum(1 for u in nbr[v] if core[u] >= core[v])
                cnt_ok &= histo[v][core[v]] == want
    return {"core": core, "init_histo": init_histo, "frontiers": frontiers,
            "iterations": len(frontiers), "cnt_ok": cnt_ok}
