#!/usr/bin/env python3
"""Benchmark of the k-core hot path on one MI355X.

One step = one full decomposition of the graph by PeelOne (Alg. 4) and one by
HistoCore (Alg. 6), both through the C ABI, inputs resident in HBM.  The
metric is coreness GTEPS: directed CSR entries |E| processed per second,
counting each of the two decompositions (2 |E| per step).  Prints one JSON
line; details of the run go to stderr.

The graph is generated on the GPU from a counter-based RNG before timing.
``--gpus`` above 1 is refused: the measurement covers a single GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_graph(name: str, device: str):
    import graphgen as gg
    if name == "er10k":
        return gg.er_10k(device=device), "ER G(n=10000, avg deg 8), seed 1, int32 CSR"
    if name == "rmat22":
        return gg.rmat22(device=device), ("RMAT scale 22, edge factor 16, (0.57,0.19,0.19,0.05), "
                                          "symmetrised, deduplicated, permuted, int32 CSR, seed 22")
    if name == "rmat26":
        return gg.rmat26_block(device=device), ("RMAT scale 26, edge factor 16 + planted block "
                                                "3000 @ p=0.6, int64 offsets, seeds 26/2601")
    raise SystemExit(f"unknown config {name}")


def algorithmic_bytes(algo: str, st: dict, n: int, m: int, w: int) -> float:
    """Bytes the method itself must move in one decomposition (w = offset width).

    PeelOne: per vertex two offset reads, core initialisation, the scan read
    that finds it, a queue push and pop, and the output write (2w + 20); per
    directed edge the column and core[u] (8); per decrement an atomic
    read-modify-write (8).
    HistoCore: InitHisto reads two offsets and writes core and reads it back
    per vertex (2w + 8), and per edge reads the column and core[u] and writes a
    bucket (12), plus the first frontier (4 each).  Each round, per frontier
    vertex: queue entry, core, buckets summed (4 each), core/oldcore/bucket
    writes, core and oldcore re-read, two offsets (28 + 2w + 4 b_v); per
    adjacency entry scanned by UpdateHisto the column and core[u] (8); per
    histogram move two atomic read-modify-writes (16); per push a queue
    write (4).  A round that rebuilds the histograms instead of UpdateHisto
    (stats "scans" counts them; each adds m to edges_scanned) moves what
    InitHisto does from the current values: two offsets and core[v] per
    vertex (2w + 4), column, core[u] and a bucket write per entry (12).
    Plus the output (4n).
    """
    if algo == "peelone":
        return n * (2 * w + 20) + 8 * m + 8 * st["atomics"]
    F, P = st["frontier_total"], st["pushes_dynamic"]
    R = st.get("scans", 0)
    init = n * (2 * w + 8) + 12 * m + 4 * (F - P)
    rounds = (F * (28 + 2 * w) + 4 * st["buckets_scanned"] + 8 * (st["edges_scanned"] - R * m)
              + 16 * st["atomics"] + 4 * P + R * (n * (2 * w + 4) + 12 * m))
    return init + rounds + 4 * n


# decomposition kernels by algorithm: grid-wide persistent, one workgroup
KERNELS = {"peelone": ("po_persistent", "po_small"), "histocore": ("hc_persistent", "hc_small")}


def coreness_properties(offsets, cols, x) -> dict:
    """Checks that hold for the coreness vector at any size, on the tensors'
    device: 0 <= x <= deg with x == 0 exactly on isolated vertices, and the
    h-index fixed point (at least x[v] neighbours valued >= x[v], at most x[v]
    valued > x[v]), which also makes {x >= k} a subgraph of minimum degree
    >= k for every k.  Returns {name: bool}."""
    import torch
    off = offsets.to(torch.int64)
    deg = off[1:] - off[:-1]
    n = deg.numel()
    xl = x.to(torch.int64)
    out = {"bounds": bool(((xl >= 0) & (xl <= deg)).all()),
           "zero_iff_isolated": bool(((xl == 0) == (deg == 0)).all())}
    ge = torch.zeros(n, dtype=torch.int64, device=x.device)
    gt = torch.zeros(n, dtype=torch.int64, device=x.device)
    chunk = 1 << 28
    for v0 in range(0, n, 1 << 22):  # rows in pieces to bound memory
        v1 = min(n, v0 + (1 << 22))
        e0, e1 = int(off[v0]), int(off[v1])
        for c0 in range(e0, e1, chunk):
            c1 = min(e1, c0 + chunk)
            pos = torch.arange(c0, c1, device=x.device)
            src = torch.searchsorted(off[v0:v1 + 1], pos, right=True) - 1 + v0
            xu = xl[cols[c0:c1].to(torch.int64)]
            xv = xl[src]
            ge.index_add_(0, src, (xu >= xv).to(torch.int64))
            gt.index_add_(0, src, (xu > xv).to(torch.int64))
    out["hindex_fixed_point"] = bool(((ge >= xl) & (gt <= xl)).all())
    return out


def host_cpu() -> str:
    """The host CPU's model name and logical CPU count, for the baseline's record."""
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, nproc={os.cpu_count()}"


def cpu_baseline(g, budget_s: float):
    import numpy as np
    import oracle
    off = g.offsets.cpu().numpy().astype(np.int64)
    cols = g.cols.cpu().numpy()
    runs, t_total, core = 0, 0.0, None
    while runs < 1 or (t_total < budget_s and runs < 5):
        t0 = time.perf_counter()
        core = oracle.bz_coreness(off, cols)
        t_total += time.perf_counter() - t0
        runs += 1
    return core, runs, t_total


def recorded_traffic(kernel: str, config: str):
    """HBM bytes per launch from the committed rocprofv3 counter summaries
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None if there is none for
    this kernel and workload or the kernel's sources changed since."""
    from paper_2402_15253_amd.profiling import recorded_traffic as rt
    return rt(kernel, config)


_COPY_GBPS = None


def achievable_gbps() -> float:
    """HBM bandwidth a plain device-to-device copy reaches on this GPU: 2^30
    bytes read and 2^30 written per copy, best of five, timed with events."""
    global _COPY_GBPS
    if _COPY_GBPS is None:
        import torch
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        best = None
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            dst.copy_(src)
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        _COPY_GBPS = 2.0 * (1 << 30) / (best / 1e3) / 1e9
        del src, dst
    return _COPY_GBPS


def _roofline(kname: str, alg_bytes: float, avg_ms: float, config: str = "") -> dict:
    gbps = alg_bytes / (avg_ms / 1e3) / 1e9
    copy = achievable_gbps()
    return {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbps / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(kname, config),
            "kernel": kname,
            "avg_launch_ms": round(avg_ms, 4), "algorithmic_bytes_per_launch": int(alg_bytes),
            "achievable_peak": round(copy, 1), "frac_achievable": round(gbps / copy, 4),
            "achievable_peak_method": "device-to-device copy of 2^30 bytes (read + write counted)"}


def random_access_roof(pico, st: dict, n: int, m: int, per_kernel: dict, ops: int = 1 << 28) -> dict:
    """The persistent kernels' times against what their random accesses
    alone cost at the rates this GPU reaches (pico_probe_random_access) over
    arrays of the sizes they touch: the per-vertex value array (4n bytes)
    and HistoCore's histogram (4m bytes).  PeelOne gathers at most one
    neighbour value per adjacency entry (batches it expands locally skip the
    read) and makes one atomic per decrement; HistoCore
    gathers one neighbour value per adjacency entry in InitHisto and in each
    round that rebuilds the histograms, and makes two atomics per histogram
    move (UpdateHisto's own value gathers, behind the neighbour-value bound,
    are left out).  `frac` is that cost over the measured launch time (1.0 =
    the launch does nothing but those accesses at the probe's rates)."""
    vals = pico.probe_random_access(4 * n, ops)
    hist = pico.probe_random_access(4 * m, ops)
    out = {"probe": {"values": vals, "histogram": hist}}
    if "po_persistent" in per_kernel and "peelone" in st:
        dec = int(st["peelone"]["atomics"])
        t = (m / vals["gathers_per_s"] + dec / vals["atomics_per_s"]) * 1e3
        avg = per_kernel["po_persistent"]["avg_ms"]
        out["po_persistent"] = {"gathers": m, "atomics": dec, "ms_at_probe_rates": round(t, 3),
                                "avg_launch_ms": avg, "frac": round(t / avg, 4)}
    if "hc_persistent" in per_kernel and "histocore" in st:
        moves = int(st["histocore"]["atomics"])
        gathers = (1 + int(st["histocore"].get("scans", 0))) * m  # InitHisto and rebuild rounds
        t = (gathers / vals["gathers_per_s"] + 2 * moves / hist["atomics_per_s"]) * 1e3
        avg = per_kernel["hc_persistent"]["avg_ms"]
        out["hc_persistent"] = {"gathers": gathers, "atomics": 2 * moves, "ms_at_probe_rates": round(t, 3),
                                "avg_launch_ms": avg, "frac": round(t / avg, 4)}
    return out


def _batch_stats_as_plain(st: dict) -> dict:
    """The batched kernel's counters under the names algorithmic_bytes reads."""
    return {"atomics": st["atomics"], "frontier_total": st["frontier_total"],
            "pushes_dynamic": st["pushes"], "buckets_scanned": st["buckets_scanned"],
            "edges_scanned": st["edges_scanned"]}


def graph_views(batch, torch):
    """Per graph of a packed batch: (offsets rebased to 0 as int64, cols view,
    n, m, first global vertex), for plain single-graph calls."""
    vptr = batch.vptr.cpu()
    e_at = batch.offsets[batch.vptr].cpu()
    views = []
    for g in range(batch.num_graphs):
        x0, x1 = int(vptr[g]), int(vptr[g + 1])
        e0, e1 = int(e_at[g]), int(e_at[g + 1])
        views.append(((batch.offsets[x0:x1 + 1] - e0).contiguous(), batch.cols[e0:e1], x1 - x0,
                      e1 - e0, x0))
    torch.cuda.synchronize()
    return views


def oracle_sample(batch, pick, budget_s: float, got=None):
    """The oracle on graphs of the batch in the order `pick`, until `budget_s`
    seconds of oracle time: (graphs done, seconds, edges, all equal to `got`)."""
    import numpy as np
    import oracle
    done, t, edges, same = 0, 0.0, 0, True
    for g in pick:
        cg = batch.graph(int(g))
        off = cg.offsets.cpu().numpy().astype(np.int64)
        cols = cg.cols.cpu().numpy()
        t0 = time.perf_counter()
        want = oracle.bz_coreness(off, cols)
        t += time.perf_counter() - t0
        done += 1
        edges += cg.m
        if got is not None:
            x0 = int(batch.vptr[int(g)])
            same = same and bool(np.array_equal(got[x0:x0 + cg.n], want))
        if t >= budget_s:
            break
    return done, t, edges, same


def bench_batched(args, pico, torch, np):
    """4,096 graphs in one batched launch per algorithm, against the plain
    method called once per graph back to back on the same stream."""
    import graphgen as gg
    dev = "cuda:0"
    t0 = time.perf_counter()
    b = gg.mixed_batch(count=args.graphs, device=dev,
                       progress=lambda g: log(f"  generating graph {g} of {args.graphs}"))
    torch.cuda.synchronize()
    G, total_n, total_m = b.num_graphs, b.total_n, b.total_m
    log(f"batch {b.name}: G={G} total_n={total_n} total_m={total_m} "
        f"generated in {time.perf_counter() - t0:.1f}s")
    order = pico.largest_first(b.vptr)
    algos = args.algos.split(",")
    views = graph_views(b, torch)
    ws_plain_bytes = max(pico.pico_workspace_bytes(v[2], v[3], pico.SINGLE_ALGOS[a] | pico.PICO_OFFSETS_I64)
                         for v in views for a in algos)
    ws_plain = torch.empty(ws_plain_bytes, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    per, outs, kern = {}, {}, {}
    for a in algos:
        code = pico.BATCH_ALGOS[a]
        tune = None
        if not args.no_tune:
            from paper_2402_15253_amd import autotune
            tune = autotune.tune_batched(b, a, order=order, log=log)
        if args.help_min is not None:
            tune = tune or pico.BatchTune()
            tune.help_min_vertices = args.help_min
        wsb = pico.pico_batched_workspace_bytes(G, total_n, total_m, code)
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        out_b = torch.empty(total_n, dtype=torch.int32, device=dev)
        st = pico.BatchStats()

        def one(stats=None):
            rc = pico.pico_coreness_batched(b.vptr, b.offsets, b.cols, G, total_n, total_m, code, order,
                                            out_b, tune, ws, wsb, stats, stream)
            if rc != pico.PICO_OK:
                raise pico.PicoError(rc, pico.pico_last_error())

        one(st)
        for _ in range(max(args.warmup - 1, 0)):
            one()
        torch.cuda.synchronize()
        pico.pico_profile_enable(not args.no_profile)
        t_start = time.perf_counter()
        for _ in range(args.steps):
            one()
        torch.cuda.synchronize()
        t_batched = (time.perf_counter() - t_start) / args.steps
        prof = pico.pico_profile_read() if not args.no_profile else {}
        pico.pico_profile_enable(False)
        # the plain method: one call per graph, back to back on the same stream
        out_p = torch.empty(total_n, dtype=torch.int32, device=dev)
        pcode = pico.SINGLE_ALGOS[a] | pico.PICO_OFFSETS_I64

        def plain_pass():
            for off, cols, n, m, x0 in views:
                if n == 0:
                    continue
                rc = pico.pico_coreness_ws(off, cols, n, m, pcode, out_p[x0:x0 + n], ws_plain,
                                           ws_plain_bytes, None, stream)
                if rc != pico.PICO_OK:
                    raise pico.PicoError(rc, pico.pico_last_error())

        if args.no_plain:
            t_plain, same = float("nan"), True
        else:
            plain_pass()  # warm-up
            torch.cuda.synchronize()
            tp0 = time.perf_counter()
            plain_pass()
            torch.cuda.synchronize()
            t_plain = time.perf_counter() - tp0
            same = bool(torch.equal(out_b, out_p))
        sd = st.as_dict()
        per[a] = {"batched_ms": round(t_batched * 1e3, 3), "plain_ms": round(t_plain * 1e3, 1),
                  "batched_graphs_per_s": round(G / t_batched, 1),
                  "plain_graphs_per_s": round(G / t_plain, 1),
                  "speedup_vs_plain": round(t_plain / t_batched, 2), "identical_to_plain": same,
                  "batched_gteps": round(total_m / t_batched / 1e9, 3),
                  "tune": tune.as_dict() if tune else None, "stats": sd}
        # (an AUTO call mixes the two algorithms' counters over two launches:
        # no single byte model, so no roofline for it)
        if "batched_kernel" in prof and a != "auto":
            launches, t_ms = prof["batched_kernel"]
            avg = t_ms / max(launches, 1)
            kern[a] = _roofline("batched_kernel", algorithmic_bytes(a, _batch_stats_as_plain(sd),
                                                                    total_n, total_m, 8), avg,
                                f"batched_{a}")
        outs[a] = out_b
        log(f"{a}: {per[a]}")
        del ws
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    value = len(algos) * G / sum(per[a]["batched_ms"] / 1e3 for a in algos)
    plain = len(algos) * G / sum(per[a]["plain_ms"] / 1e3 for a in algos)
    roof = max(kern.values(), key=lambda r: r["avg_launch_ms"]) if kern else None
    props = {}
    for a in algos:
        props[f"{a}==plain"] = per[a]["identical_to_plain"]
    if len(algos) == 2:
        props["peelone==histocore"] = bool(torch.equal(outs["peelone"], outs["histocore"]))
    cpu = None
    if args.cpu_budget > 0:
        pick = torch.randperm(G, generator=torch.Generator().manual_seed(5)).tolist()
        got = next(iter(outs.values())).cpu().numpy()
        done, t_cpu, edges, same = oracle_sample(b, pick, args.cpu_budget, got)
        props["sample==oracle"] = same
        cpu = {"value": round(done / t_cpu, 2), "unit": "graphs/s", "cores": 1, "kind": "oracle",
               "sample": f"Batagelj-Zaversnik peel, single thread, {done} graphs of the batch in a "
                         f"seeded random order ({edges} directed edges, {t_cpu:.1f}s); host {host_cpu()}"}
    ok = all(props.values())
    if not ok:
        log(f"PARITY FAILURE: {props}")
    rec = {
        "metric": "batched graphs/s (one launch per algorithm) vs sequential plain launches",
        "value": round(value, 1), "unit": "graphs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(sum(per[a]["batched_ms"] for a in algos), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{G} graphs, vertex counts log-uniform in [200, 200000], even ones "
                               "Erdos-Renyi G(n, M) avg degree U(4,32), odd ones R-MAT edge factor "
                               "U(8,16); packed multi-CSR, int64 offsets, int32 graph-local cols; "
                               "seed 4096",
                   "graphs": G, "total_n": total_n, "total_m": total_m,
                   "step": " + ".join(f"batched {a}" for a in algos), "parallelism": "single GPU"},
        "plain_graphs_per_s": round(plain, 1), "vs_plain": round(value / plain, 2),
        "roofline": roof, "cpu_baseline": cpu, "per_algo": per,
        "parity": "identical to plain calls" + (" and oracle sample" if cpu else "") if ok else props,
    }
    print(json.dumps(rec), flush=True)
    if not ok:
        sys.exit(1)


def bench_serving(args, pico, torch, np):
    """A Poisson stream of requests served by the continuous-batching server,
    then the same trace through a serial loop of plain calls."""
    import graphgen as gg
    dev = "cuda:0"
    algo = args.algos.split(",")[0]
    code = pico.ALGOS[algo]
    t0 = time.perf_counter()
    pool = gg.serving_pool(count=args.pool, device=dev,
                           progress=lambda g: log(f"  generating pool graph {g} of {args.pool}"))
    torch.cuda.synchronize()
    log(f"pool {pool.name}: total_n={pool.total_n} total_m={pool.total_m} "
        f"in {time.perf_counter() - t0:.1f}s")
    arrivals, pick = gg.poisson_trace(args.rate, args.duration, pool.num_graphs)
    R = arrivals.numel()
    views = graph_views(pool, torch)
    # each pool graph alone (the plain single-graph call): the reference
    ws_bytes = max(pico.pico_workspace_bytes(v[2], v[3], code | pico.PICO_OFFSETS_I64) for v in views)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    ref = torch.empty(pool.total_n, dtype=torch.int32, device=dev)
    plain_ms = []
    for off, cols, n, m, x0 in views:
        st = pico.PicoStats()
        rc = pico.pico_coreness_ws(off, cols, n, m, code | pico.PICO_OFFSETS_I64, ref[x0:x0 + n], ws,
                                   ws_bytes, st, None)
        if rc != pico.PICO_OK:
            raise pico.PicoError(rc, pico.pico_last_error())
        plain_ms.append(st.elapsed_ms)
    vp = pool.vptr.cpu().numpy()
    ep = pool.offsets[pool.vptr].cpu().numpy()
    sizes = vp[1:] - vp[:-1]
    medges = ep[1:] - ep[:-1]
    req_n = sizes[pick.numpy()]
    base = np.concatenate([[0], np.cumsum(req_n)])
    out = torch.full((int(base[-1]) + 1,), -1, dtype=torch.int32, device=dev)  # -1: never written
    off_ptr = [pool.offsets.data_ptr() + 8 * int(vp[g]) for g in range(pool.num_graphs)]
    cols_ptr = pool.cols.data_ptr()
    out_ptr = out.data_ptr()
    free = torch.cuda.mem_get_info()[0]
    arena = int(min(args.arena_gb * 1e9, free - (8 << 30))) & ~255
    log(f"requests {R} over {args.duration}s; arena {arena / 1e9:.1f} GB; "
        f"pool graph sizes p50 {np.median(sizes):.0f} p99 {np.percentile(sizes, 99):.0f}")
    tune = None
    if not args.no_tune:
        from paper_2402_15253_amd import autotune
        tune = autotune.tune_batched(pool, algo, order=pico.largest_first(pool.vptr), log=log)
    srv = pico.Server(algo, arena_bytes=arena, max_inflight=args.inflight,
                      max_tasks_per_launch=4096, tune=tune)
    torch.cuda.synchronize()
    arr = arrivals.numpy()
    pk = pick.numpy()
    t_done = np.zeros(R)
    t_start = time.perf_counter_ns()
    i = done = 0
    last_log = time.perf_counter()
    while done < R:
        now = (time.perf_counter_ns() - t_start) / 1e9
        while i < R and arr[i] <= now:
            g = int(pk[i])
            srv.submit_ptrs(off_ptr[g], cols_ptr, int(sizes[g]), int(medges[g]),
                            out_ptr + 4 * int(base[i]), i)
            i += 1
        k, buf = srv.progress_raw()
        if k:
            seen = (time.perf_counter_ns() - t_start) / 1e9  # result ready, as the client sees it
            for j in range(k):
                t_done[buf[j].tag] = seen
        done += k
        if time.perf_counter() - last_log > 10:
            last_log = time.perf_counter()
            log(f"  t={now:.1f}s submitted {i} done {done} {srv.status()}")
    st = srv.status()
    srv.close()
    elapsed = t_done.max()
    lat = (t_done - arr) * 1e3
    served = {"graphs_per_s": round(R / elapsed, 1), "p50_ms": round(float(np.percentile(lat, 50)), 3),
              "p99_ms": round(float(np.percentile(lat, 99)), 3),
              "max_ms": round(float(lat.max()), 3), "launches": st["launches"],
              "requests": R, "elapsed_s": round(float(elapsed), 3)}
    log(f"server: {served}")
    # every request's result equals its graph's result alone
    same = True
    for r in range(R):
        g = int(pk[r])
        got, want = out[base[r]:base[r + 1]], ref[vp[g]:vp[g + 1]]
        if not torch.equal(got, want):
            same = False
            bad = torch.nonzero(got != want).flatten()
            ex = [(int(v), int(got[v]), int(want[v])) for v in bad[:6].tolist()]
            log(f"request {r} (graph {g}, n={int(sizes[g])}, arrival {arr[r]:.3f}s) differs from the "
                f"graph alone at {bad.numel()} vertices ({int((got[bad] == -1).sum())} never written); "
                f"(vertex, served, alone): {ex}")
            break
    # the serial plain loop on the same trace (capped in wall time)
    ws_stream = torch.cuda.current_stream()
    done_p = np.full(R, np.nan)
    t_start = time.perf_counter()
    for r in range(R):
        now = time.perf_counter() - t_start
        if now > args.plain_budget:
            break
        if arr[r] > now:
            time.sleep(arr[r] - now)
        off, cols, n, m, x0 = views[int(pk[r])]
        rc = pico.pico_coreness_ws(off, cols, n, m, code | pico.PICO_OFFSETS_I64,
                                   out[base[r]:base[r] + n], ws, ws_bytes, None, ws_stream)
        if rc != pico.PICO_OK:
            raise pico.PicoError(rc, pico.pico_last_error())
        done_p[r] = time.perf_counter() - t_start
    fin = ~np.isnan(done_p)
    lat_p = (done_p[fin] - arr[fin]) * 1e3
    plain = {"graphs_per_s": round(float(fin.sum() / np.nanmax(done_p)), 1),
             "p50_ms": round(float(np.percentile(lat_p, 50)), 3),
             "p99_ms": round(float(np.percentile(lat_p, 99)), 3),
             "completed": int(fin.sum()), "of": R,
             "note": "stopped at the wall-clock cap" if fin.sum() < R else "whole trace"}
    log(f"plain loop: {plain}")
    cpu = None
    if args.cpu_budget > 0:
        done_c, t_cpu, edges, _ = oracle_sample(pool, pk.tolist(), args.cpu_budget)
        cpu = {"value": round(done_c / t_cpu, 2), "unit": "graphs/s", "cores": 1, "kind": "oracle",
               "sample": f"Batagelj-Zaversnik peel, single thread, the first {done_c} requests' "
                         f"graphs ({edges} directed edges, {t_cpu:.1f}s); host {host_cpu()}"}
    rec = {
        "metric": "served graphs/s with p50/p99 latency (arrival to result) vs a serial plain loop",
        "value": served["graphs_per_s"], "unit": "graphs/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(float(elapsed) * 1e3, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"Poisson arrivals {args.rate:g}/s for {args.duration:g}s, graphs "
                               f"from a pool of {pool.num_graphs} R-MAT (edge factor 16) graphs with "
                               "lognormal vertex counts (median 20000, sigma 1.5, cap 8M); seeds 2000",
                   "algo": algo, "requests": R, "arena_bytes": arena,
                   "inflight_slots": args.inflight, "parallelism": "single GPU"},
        "latency_ms": {"p50": served["p50_ms"], "p99": served["p99_ms"], "max": served["max_ms"]},
        "served": served, "plain_loop": plain,
        "vs_plain": round(served["graphs_per_s"] / max(plain["graphs_per_s"], 1e-9), 2),
        "roofline": None, "cpu_baseline": cpu,
        "parity": "every request identical to its graph alone" if same else "MISMATCH",
        "pool_plain_ms_mean": round(float(np.mean(plain_ms)), 3),
    }
    print(json.dumps(rec), flush=True)
    if not same:
        sys.exit(1)


def bench_update(args, pico, torch, np):
    """Core maintenance on RMAT-22: the coreness after deleting 0.1% of the
    undirected edges (and, second, after inserting 16 edges), by HistoCore
    started from the old coreness (pico_coreness_update), against cold
    HistoCore and PeelOne on the changed graph."""
    import graphgen as gg
    dev = "cuda:0"
    t0 = time.perf_counter()
    g = gg.rmat22(device=dev)
    old = pico.coreness(g.offsets, g.cols, "peelone")
    cases = {}
    for name, frac, ins in (("delete 0.1%", 0.001, 0), ("insert 16", 0.0, 16)):
        h, b = gg.edit_edges(g, frac, ins, 2201)
        cases[name] = (h, b)
    torch.cuda.synchronize()
    log(f"RMAT-22 n={g.n} m={g.m}; edits generated in {time.perf_counter() - t0:.1f}s")
    code_hc = pico.algo_code("histocore", g.offsets)
    ws_bytes = max(pico.pico_workspace_bytes(h.n, h.m, code_hc) for h, _ in cases.values())
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    w = 8 if g.offsets.dtype == torch.int64 else 4
    per, first = {}, None
    for name, (h, b) in cases.items():
        out = torch.empty(h.n, dtype=torch.int32, device=dev)
        st = pico.PicoStats()

        def update():
            rc = pico.pico_coreness_update(h.offsets, h.cols, h.n, h.m, code_hc, old, b, out, ws, ws_bytes,
                                           st, None)
            if rc != pico.PICO_OK:
                raise pico.PicoError(rc, pico.pico_last_error())

        for _ in range(args.warmup):
            update()
        torch.cuda.synchronize()
        pico.pico_profile_enable(not args.no_profile)
        tw = time.perf_counter()
        for _ in range(args.steps):
            update()
        torch.cuda.synchronize()
        el = (time.perf_counter() - tw) / args.steps
        prof = pico.pico_profile_read() if not args.no_profile else {}
        pico.pico_profile_enable(False)
        sd = st.as_dict()
        cold_hc, st_hc = pico.coreness(h.offsets, h.cols, "histocore", workspace=ws, with_stats=True)
        cold_po, st_po = pico.coreness(h.offsets, h.cols, "peelone", with_stats=True)
        ok = bool(torch.equal(out, cold_po)) and bool(torch.equal(cold_hc, cold_po))
        props = coreness_properties(h.offsets, h.cols, out)
        ok = ok and all(props.values())
        rec = {"inserted": b, "m": h.m, "update_ms": round(el * 1e3, 3),
               "update_rounds": sd["iterations"], "update_frontier_total": sd["frontier_total"],
               "cold_histocore_ms": round(st_hc["elapsed_ms"], 3), "cold_histocore_rounds": st_hc["iterations"],
               "cold_histocore_frontier_total": st_hc["frontier_total"],
               "cold_peelone_ms": round(st_po["elapsed_ms"], 3), "identical_to_cold": ok}
        if "hc_persistent" in prof:
            launches, t_ms = prof["hc_persistent"]
            avg = t_ms / launches
            rec["roofline"] = _roofline("hc_persistent", algorithmic_bytes("histocore", sd, h.n, h.m, w), avg,
                                        "rmat22-update")
        per[name] = rec
        log(f"{name}: {rec}")
        if first is None:
            first = (name, h, rec)
    name, h, rec = first
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cpu = None
    if args.cpu_budget > 0:
        want, runs, t_cpu = cpu_baseline(h, args.cpu_budget)
        cpu = {"value": round(h.m * runs / t_cpu / 1e9, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"Batagelj-Zaversnik peel from scratch on the changed RMAT-22 ({name}), single "
                         f"thread, {runs} run(s), {t_cpu:.1f}s"}
        got = pico.coreness(h.offsets, h.cols, "peelone").cpu().numpy()
        per[name]["identical_to_oracle"] = bool(np.array_equal(got, want))
    ok = all(r["identical_to_cold"] and r.get("identical_to_oracle", True) for r in per.values())
    out = {
        "metric": "core maintenance GTEPS (|E| of the changed graph / update time)",
        "value": round(h.m / (rec["update_ms"] / 1e3) / 1e9, 4), "unit": "GTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": rec["update_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "RMAT-22 (scale 22, edge factor 16, seed 22, int32 CSR); each undirected "
                               "edge deleted with probability 0.001 (seed 2201); HistoCore from the old "
                               "coreness; second case: 16 random insertions, bound old + 16",
                   "parallelism": "single GPU"},
        "roofline": rec.get("roofline"), "cpu_baseline": cpu, "cases": per,
        "parity": "identical to cold PeelOne and HistoCore" + (" and the oracle" if cpu else "")
                  if ok else "MISMATCH",
    }
    print(json.dumps(out), flush=True)
    if not ok:
        sys.exit(1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="rmat26",
                    choices=["er10k", "rmat22", "rmat26", "batched", "serving", "rmat22-update"])
    ap.add_argument("--cpu-budget", type=float, default=12.0,
                    help="seconds of oracle time for the CPU baseline (0 = skip)")
    ap.add_argument("--algos", default="peelone,histocore",
                    help="comma list of algorithms per step (the metric uses both)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, copy 1 GiB device to device (HBM counter calibration)")
    ap.add_argument("--no-profile", action="store_true",
                    help="do not bracket kernels with HIP events during the timed steps")
    ap.add_argument("--no-ablations", action="store_true",
                    help="single graphs: skip the PeelOne ablation runs after the timed steps")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched: skip the autotuner and use the default launch parameters")
    ap.add_argument("--graphs", type=int, default=4096, help="batched: number of graphs")
    ap.add_argument("--help-min", type=int, default=None,
                    help="batched: vertices from which a graph takes helpers (-1 never; default: the "
                         "library's or the autotuner's)")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched: skip the per-graph plain-call comparison (profiling runs)")
    ap.add_argument("--rate", type=float, default=2000.0, help="serving: requests per second")
    ap.add_argument("--duration", type=float, default=60.0, help="serving: trace length (s)")
    ap.add_argument("--pool", type=int, default=2048, help="serving: graphs in the request pool")
    ap.add_argument("--arena-gb", type=float, default=200.0,
                    help="serving: HBM admission budget for request state (GB)")
    ap.add_argument("--inflight", type=int, default=4, help="serving: launch slots")
    ap.add_argument("--plain-budget", type=float, default=60.0,
                    help="serving: wall-clock cap (s) on the serial plain-loop baseline")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU; runs on several GPUs are not implemented "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2402_15253_amd as pico

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.config == "batched":
        return bench_batched(args, pico, torch, np)
    if args.config == "serving":
        return bench_serving(args, pico, torch, np)
    if args.config == "rmat22-update":
        return bench_update(args, pico, torch, np)
    t0 = time.perf_counter()
    g, desc = make_graph(args.config, dev)
    torch.cuda.synchronize()
    log(f"graph {g.name}: n={g.n} m={g.m} generated in {time.perf_counter() - t0:.1f}s")
    n, m = g.n, g.m
    w = 8 if g.offsets.dtype == torch.int64 else 4
    algos = {a: pico.algo_code(a, g.offsets) for a in args.algos.split(",")}
    ws_bytes = max(pico.pico_workspace_bytes(n, m, a) for a in algos.values())
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    outs = {k: torch.empty(n, dtype=torch.int32, device=dev) for k in algos}
    stream = torch.cuda.current_stream()
    stats = {k: pico.PicoStats() for k in algos}

    def step():
        for name, a in algos.items():
            rc = pico.pico_coreness_ws(g.offsets, g.cols, n, m, a, outs[name], ws, ws_bytes,
                                       stats[name], stream)
            if rc != pico.PICO_OK:
                raise pico.PicoError(rc, pico.pico_last_error())

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    pico.pico_profile_enable(not args.no_profile)
    per_algo_ms = {k: 0.0 for k in algos}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
        for k in algos:
            per_algo_ms[k] += stats[k].elapsed_ms
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = pico.pico_profile_read() if not args.no_profile else {}
    pico.pico_profile_enable(False)
    ms_per_step = elapsed / args.steps * 1e3
    value = len(algos) * m * args.steps / elapsed / 1e9

    st = {k: stats[k].as_dict() for k in algos}
    log(json.dumps({"stats": st}))
    log("kernel times over the timed steps (launches, total ms):")
    for name, (cnt, tot) in sorted(prof.items(), key=lambda x: -x[1][1]):
        log(f"  {name:18s} {cnt:8d} {tot:10.3f}")

    # Roofline of the kernel that takes the most time: one persistent launch
    # per decomposition, timed with HIP events on the call's stream.
    roofline, per_kernel = None, {}
    for algo, knames in KERNELS.items():
        for kname in knames:
            if kname not in prof or algo not in st:
                continue
            launches, t_ms = prof[kname]
            b = algorithmic_bytes(algo, st[algo], n, m, w)
            avg_s = t_ms / launches / 1e3
            per_kernel[kname] = {"launches": launches, "avg_ms": round(t_ms / launches, 4),
                                 "alg_bytes": int(b), "alg_GBps": round(b / avg_s / 1e9, 1)}
    if per_kernel:
        kname = max(per_kernel, key=lambda k: per_kernel[k]["avg_ms"] * per_kernel[k]["launches"])
        pk = per_kernel[kname]
        roofline = _roofline(kname, pk["alg_bytes"], pk["avg_ms"], args.config)
    random_access = random_access_roof(pico, st, n, m, per_kernel) if per_kernel else None
    if random_access:
        log(f"random-access roof: {json.dumps(random_access)}")

    # Ablations of PeelOne (outside the timed region): what the dynamic
    # frontier and the assertion decrement save (Tables IV and V).
    ablations = None
    if not args.no_ablations and "peelone" in algos:
        ablations = {}
        for variant in ("peelone", "peelone-static", "peelone-rollback", "gpp"):
            code = pico.algo_code(variant, g.offsets)
            vout = torch.empty(n, dtype=torch.int32, device=dev)
            vst = pico.PicoStats()
            times = []
            for _ in range(3):
                rc = pico.pico_coreness_ws(g.offsets, g.cols, n, m, code, vout, ws, ws_bytes, vst, stream)
                if rc != pico.PICO_OK:
                    raise pico.PicoError(rc, pico.pico_last_error())
                times.append(vst.elapsed_ms)
            ablations[variant] = {"ms": round(min(times), 3), "iterations": vst.iterations,
                                  "atomics": vst.atomics, "pushes_dynamic": vst.pushes_dynamic,
                                  "identical": bool(torch.equal(vout, outs["peelone"]))}
        # Index2core baselines against HistoCore (Table VI): same rounds,
        # every h-index rebuilt from the neighbours
        i2c_bytes = max(pico.pico_workspace_bytes(n, m, pico.algo_code(v, g.offsets))
                        for v in ("cntcore", "nbrcore"))
        i2c_ws = torch.empty(max(i2c_bytes, ws_bytes), dtype=torch.uint8, device=dev)
        for variant in ("histocore", "cntcore", "nbrcore"):
            code = pico.algo_code(variant, g.offsets)
            vout = torch.empty(n, dtype=torch.int32, device=dev)
            vst = pico.PicoStats()
            times = []
            for _ in range(2):
                rc = pico.pico_coreness_ws(g.offsets, g.cols, n, m, code, vout, i2c_ws, i2c_ws.numel(), vst,
                                           stream)
                if rc != pico.PICO_OK:
                    raise pico.PicoError(rc, pico.pico_last_error())
                times.append(vst.elapsed_ms)
            ablations[variant] = {"ms": round(min(times), 3), "iterations": vst.iterations,
                                  "hindex_computed": vst.frontier_total, "edges_scanned": vst.edges_scanned,
                                  "atomics": vst.atomics,
                                  "identical": bool(torch.equal(vout, outs["peelone"]))}
        del i2c_ws
        log(f"ablations: {ablations}")

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # Parity: properties at any size on the GPU, plus PeelOne == HistoCore;
    # the CPU baseline leg also compares with the oracle it times.
    props = {}
    for k in algos:
        for name, ok in coreness_properties(g.offsets, g.cols, outs[k]).items():
            props[f"{k}:{name}"] = ok
    if len(algos) == 2:
        props["peelone==histocore"] = bool(torch.equal(outs["peelone"], outs["histocore"]))
    if ablations:
        for variant, rec in ablations.items():
            props[f"{variant}==peelone"] = rec["identical"]
    want = None
    cpu = None
    if args.cpu_budget > 0:
        want, runs, t_cpu = cpu_baseline(g, args.cpu_budget)
        cpu = {"value": round(m * runs / t_cpu / 1e9, 4), "unit": "GTEPS", "cores": 1,
               "kind": "oracle",
               "sample": f"Batagelj-Zaversnik peel (the oracle), single thread, whole {args.config} "
                         f"graph ({m} directed entries), {runs} run(s), {t_cpu:.1f}s; host {host_cpu()}"}
    parity = dict(props)
    if want is not None:
        for k in algos:
            parity[f"{k}==oracle"] = bool(np.array_equal(outs[k].cpu().numpy(), want))
    if not all(parity.values()):
        log(f"PARITY FAILURE: {parity}")

    rec = {
        "metric": "coreness GTEPS (|E|/s) + %HBM peak",
        "value": round(value, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "m": m, "step": " + ".join(algos) + ", one each",
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "random_access": random_access,
        "cpu_baseline": cpu,
        "per_algo_ms": {k: round(v / args.steps, 3) for k, v in per_algo_ms.items()},
        "per_algo_gteps": {k: round(m / (v / args.steps / 1e3) / 1e9, 3)
                           for k, v in per_algo_ms.items()},
        "kernels": per_kernel,
        "ablations": ablations,
        "levels_l1": st.get("peelone", {}).get("iterations"),
        "rounds_l2": st.get("histocore", {}).get("iterations"),
        "k_max": int(next(iter(outs.values())).max().item()) if n else 0,
        "parity": ("bit-exact vs oracle" if want is not None else "properties") if all(parity.values())
                  else parity,
    }
    print(json.dumps(rec), flush=True)
    if not all(parity.values()):
        sys.exit(1)


if __name__ == "__main__":
    main()
