"""Autotuner of the batched kernel's launch parameters.

The batched kernel (``pico_coreness_batched`` / ``pico_coreness_tasks``) has
three knobs, all in ``pico_batch_tune``:

* ``lds_bytes``: the LDS tier.  A graph whose vertex values fit keeps them in
  the workgroup's LDS (LDS atomics for the decrements and reads), larger ones
  in global memory.  More LDS per workgroup means fewer workgroups per
  compute unit.
* ``blocks_per_cu``: resident workgroups per compute unit (graphs in flight
  per CU), up to what registers and LDS allow.
* ``sum_wave_min`` (HistoCore): values above it scan their histogram buckets
  with a whole wave in SumHisto, smaller ones with one thread.

The tuner times every candidate on the batch it is given (each candidate's
result is checked against the first one's: the output is unique, so any
difference is a bug), keeps the fastest, and caches the choice per device,
algorithm and batch shape in a JSON file.
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import (BATCH_ALGOS, BatchStats, BatchTune, PicoError, PICO_OK, pico_batched_workspace_bytes,
               pico_coreness_batched, pico_last_error)
from .profiling import source_hash

CACHE = os.environ.get("PICO_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "pico", "batched_tune.json"))

LDS_CANDIDATES = (0, 16 * 1024, 32 * 1024, 64 * 1024, 96 * 1024)
BLOCKS_CANDIDATES = (0, 1, 2, 4, 8)
SUM_WAVE_CANDIDATES = (32, 64, 128)


def _key(batch, algo: str) -> str:
    p = torch.cuda.get_device_properties(batch.offsets.device)
    n, m, G = batch.offsets.numel() - 1, batch.cols.numel(), batch.vptr.numel() - 1
    # shape class: graph count and mean sizes to two significant digits
    def sig(x):
        return f"{float(x):.2g}"
    # the kernel's sources too: a choice timed on another revision is not reused
    return (f"{p.name}|{p.multi_processor_count}|{algo}|G{sig(G)}|n{sig(n / max(G, 1))}"
            f"|m{sig(m / max(G, 1))}|{source_hash('batched_kernel')}")


def _load() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict) -> None:
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + f".{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def tune_batched(batch, algo: str, *, order=None, reps: int = 2, use_cache: bool = True,
                 log=None) -> BatchTune:
    """Fastest BatchTune for this batch (device-resident) and algorithm:
    LDS tier and workgroups per CU first, then (HistoCore) the SumHisto wave
    threshold at the best of those, then whether large graphs take helpers
    (the library default, or never)."""
    key = _key(batch, algo)
    cache = _load() if use_cache else {}
    if key in cache:
        c = cache[key]
        if log:
            log(f"autotune {algo}: cached {c}")
        return BatchTune(c["lds_bytes"], c["blocks_per_cu"], c["sum_wave_min"], c.get("help_min_vertices", 0))
    code = BATCH_ALGOS[algo]
    G = batch.vptr.numel() - 1
    n, m = batch.offsets.numel() - 1, batch.cols.numel()
    wsb = pico_batched_workspace_bytes(G, n, m, code)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=batch.offsets.device)
    out = torch.empty(max(n, 1), dtype=torch.int32, device=batch.offsets.device)
    stream = torch.cuda.current_stream()
    state = {"ref": None, "seen": {}}

    def measure(t: BatchTune):
        st = BatchStats()
        rc = pico_coreness_batched(batch.vptr, batch.offsets, batch.cols, G, n, m, code, order, out,
                                   t, ws, wsb, st, stream)
        if rc != PICO_OK:
            raise PicoError(rc, pico_last_error())
        eff = (st.lds_bytes, st.blocks_per_cu, t.sum_wave_min, t.help_min_vertices)
        if eff in state["seen"]:  # clamped to a configuration already timed
            return state["seen"][eff]
        if state["ref"] is None:
            state["ref"] = out.clone()
        elif not torch.equal(out, state["ref"]):
            raise RuntimeError(f"batched result differs under tune {t.as_dict()}")
        t0 = time.perf_counter()
        for _ in range(reps):
            rc = pico_coreness_batched(batch.vptr, batch.offsets, batch.cols, G, n, m, code, order,
                                       out, t, ws, wsb, None, stream)
            if rc != PICO_OK:
                raise PicoError(rc, pico_last_error())
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        state["seen"][eff] = dt
        if log:
            log(f"autotune {algo}: lds {eff[0]} blocks/CU {eff[1]} sum_wave_min {eff[2]} "
                f"help_min {eff[3]}: {dt * 1e3:.2f} ms")
        return dt

    best, best_t = None, float("inf")
    for lds in LDS_CANDIDATES:
        for bpc in BLOCKS_CANDIDATES:
            t = BatchTune(lds, bpc, 0)
            dt = measure(t)
            if dt < best_t:
                best, best_t = t, dt
    if algo in ("histocore", "auto"):
        base = best
        for sw in SUM_WAVE_CANDIDATES:
            t = BatchTune(base.lds_bytes, base.blocks_per_cu, sw)
            dt = measure(t)
            if dt < best_t:
                best, best_t = t, dt
    # helpers bound the time of a launch's largest graphs, but cost a little
    # throughput when the launch is busy anyway
    t = BatchTune(best.lds_bytes, best.blocks_per_cu, best.sum_wave_min, -1)
    dt = measure(t)
    if dt < best_t:
        best, best_t = t, dt
    cache = _load() if use_cache else {}
    cache[key] = dict(best.as_dict(), ms=round(best_t * 1e3, 3))
    if use_cache:
        _store(cache)
    if log:
        log(f"autotune {algo}: chose {best.as_dict()} ({best_t * 1e3:.2f} ms)")
    return best
