"""Host-side checks of the C ABI: the library builds, loads and exports every
entry point that include/pico.h declares; argument checks that need no GPU."""
import ctypes
import os
import re

import pytest
import torch

import paper_2402_15253_amd as pico

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "pico.h")) as f:
        text = f.read()
    return re.findall(r"PICO_API\s+[\w\s\*]+?\b(pico_\w+)\s*\(", text)


def test_header_declares_the_python_names():
    names = _declared()
    assert set(names) == set(pico.EXPORTED_SYMBOLS)
    for name in names:
        assert callable(getattr(pico, name))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(pico.library_path())
    for name in _declared():
        assert hasattr(lib, name), name


def test_workspace_and_status_without_gpu():
    assert pico.pico_workspace_bytes(0, 0, pico.PICO_ALGO_PEELONE) >= 0
    a = pico.pico_workspace_bytes(1000, 8000, pico.PICO_ALGO_PEELONE)
    b = pico.pico_workspace_bytes(1000, 8000, pico.PICO_ALGO_HISTOCORE)
    assert a >= 4 * 4000 and b >= 4 * 8000
    with pytest.raises(pico.PicoError):
        pico.pico_workspace_bytes(-1, 0, pico.PICO_ALGO_PEELONE)
    with pytest.raises(pico.PicoError):
        pico.pico_workspace_bytes(10, 2**31, pico.PICO_ALGO_PEELONE)  # needs int64 offsets
    assert pico.pico_workspace_bytes(10, 2**31, pico.PICO_ALGO_PEELONE | pico.PICO_OFFSETS_I64) > 0
    assert pico.pico_status_string(pico.PICO_EINVAL) == "invalid argument"
    assert "gfx950" in pico.pico_version()


def test_argument_errors_need_no_device():
    # rejected before any device work
    assert pico.pico_coreness(None, None, -5, 0, 0, None) == pico.PICO_EINVAL
    assert pico.pico_coreness(None, None, 10, 0, 0, None) == pico.PICO_EINVAL
    assert "NULL" in pico.pico_last_error()
    assert pico.pico_coreness(None, None, 0, 0, 7, None) == pico.PICO_EINVAL
    assert pico.pico_coreness(None, None, 0, 0, 0, None) == pico.PICO_OK  # n == 0: no-op
    assert pico.pico_coreness_ws(None, None, 0, 0, 1, None, None, 0) == pico.PICO_OK
    # path flags: one at a time, single-graph calls only
    both = pico.PICO_PATH_GRID | pico.PICO_PATH_WG
    assert pico.pico_coreness(None, None, 0, 0, both, None) == pico.PICO_EINVAL
    assert "exclusive" in pico.pico_last_error()
    assert pico.pico_coreness(None, None, 0, 0, pico.PICO_PATH_WG, None) == pico.PICO_OK
    assert pico.pico_coreness(None, None, 0, 0, 0x4000, None) == pico.PICO_EINVAL
    # PeelOne ablations: one at a time, PeelOne only, grid path only
    po, hc_ = pico.PICO_ALGO_PEELONE, pico.PICO_ALGO_HISTOCORE
    st_, rb = pico.PICO_PO_STATIC, pico.PICO_PO_ROLLBACK
    assert pico.pico_coreness(None, None, 0, 0, po | st_ | rb, None) == pico.PICO_EINVAL
    assert pico.pico_coreness(None, None, 0, 0, hc_ | st_, None) == pico.PICO_EINVAL
    assert pico.pico_coreness(None, None, 0, 0, po | rb | pico.PICO_PATH_WG, None) == pico.PICO_ENOTSUP
    assert pico.pico_coreness(None, None, 0, 0, po | st_, None) == pico.PICO_OK
    assert pico.algo_code("peelone-static", torch.zeros(1, dtype=torch.int64)) == (
        po | st_ | pico.PICO_OFFSETS_I64)
    # algorithm choice: PICO_ALGO_AUTO only; n == 0 picks PeelOne without device work
    rc, chosen, feat = pico.pico_select_algorithm(None, None, 0, 0, pico.PICO_ALGO_AUTO, None, 0)
    assert (rc, chosen, feat) == (pico.PICO_OK, pico.PICO_ALGO_PEELONE, [0, 0, 0])
    assert pico.pico_select_algorithm(None, None, 0, 0, pico.PICO_ALGO_PEELONE, None, 0)[0] == pico.PICO_EINVAL
    assert pico.pico_coreness(None, None, 0, 0, pico.PICO_ALGO_AUTO, None) == pico.PICO_OK
    assert pico.pico_workspace_bytes(1000, 8000, pico.PICO_ALGO_AUTO) >= max(
        pico.pico_workspace_bytes(1000, 8000, a) for a in (pico.PICO_ALGO_PEELONE, pico.PICO_ALGO_HISTOCORE))
    # random-access probe: argument checks come before any device call
    assert pico.pico_probe_random_access(None, 1 << 20, 1000)[0] == pico.PICO_EINVAL
    assert pico.pico_probe_random_access(None, 0, 1000)[0] == pico.PICO_EINVAL
    # Index2core baselines: grid path only
    for alg in (pico.PICO_ALGO_CNTCORE, pico.PICO_ALGO_NBRCORE):
        assert pico.pico_coreness(None, None, 0, 0, alg | pico.PICO_PATH_WG, None) == pico.PICO_ENOTSUP
        assert pico.pico_workspace_bytes(1000, 8000, alg) >= pico.pico_workspace_bytes(1000, 8000, hc_)
    # core maintenance: HistoCore only, bounds required, bound_add >= 0
    up = pico.pico_coreness_update
    hc = pico.PICO_ALGO_HISTOCORE
    assert up(None, None, 0, 0, pico.PICO_ALGO_PEELONE, None, 0, None, None, 0) == pico.PICO_ENOTSUP
    assert up(None, None, 0, 0, hc, None, -1, None, None, 0) == pico.PICO_EINVAL
    assert up(None, None, 10, 0, hc, None, 0, None, None, 0) == pico.PICO_EINVAL
    assert "prev_core" in pico.pico_last_error()
    assert up(None, None, 0, 0, hc, None, 0, None, None, 0) == pico.PICO_OK  # n == 0: no-op
    # a workspace sized without a path flag serves either path
    for algo in (pico.PICO_ALGO_PEELONE, pico.PICO_ALGO_HISTOCORE):
        auto = pico.pico_workspace_bytes(5000, 40000, algo)
        assert auto == pico.pico_workspace_bytes(5000, 40000, algo | pico.PICO_PATH_GRID)
        assert auto == pico.pico_workspace_bytes(5000, 40000, algo | pico.PICO_PATH_WG)


def test_task_and_server_argument_checks_need_no_device():
    pe, hc = pico.PICO_ALGO_PEELONE, pico.PICO_ALGO_HISTOCORE
    # per-task scratch: four int32 arrays of n (PeelOne), plus oldcore n and histogram m
    assert pico.pico_task_scratch_bytes(1000, 8000, pe) == 4 * 1024 * 4
    assert pico.pico_task_scratch_bytes(1000, 8000, hc) == (5 * 1024 + 8000) * 4
    assert pico.pico_task_scratch_bytes(0, 0, pe) == 0
    with pytest.raises(pico.PicoError):
        pico.pico_task_scratch_bytes(2**31, 0, pe)
    assert pico.pico_tasks_workspace_bytes(100) > 100 * ctypes.sizeof(pico.Task)
    assert ctypes.sizeof(pico.Task) == 56 and ctypes.sizeof(pico.BatchTune) == 16
    assert ctypes.sizeof(pico.BatchStats) == 9 * 8 + 8 + 3 * 8
    assert ctypes.sizeof(pico.Completion) == 40
    # bad task lists are rejected on the host, before any device work
    bad = pico.Task(None, None, -1, 0, None, None, 0)
    assert pico.pico_coreness_tasks([bad], pe, None, None, 0) == pico.PICO_EINVAL
    assert "task 0" in pico.pico_last_error()
    short = pico.Task(1, 1, 10, 40, 1, 256, 100)  # scratch too small: never dereferenced
    assert pico.pico_coreness_tasks([short], pe, None, None, 0) == pico.PICO_ENOMEM
    assert pico.pico_coreness_tasks([], pe, None, None, 0) == pico.PICO_OK
    tune = pico.BatchTune()
    tune.help_min_vertices = -5
    assert pico.pico_coreness_tasks([], pe, tune, None, 0) == pico.PICO_EINVAL
    # server configuration errors come before the device check
    cfg = pico.ServerConfig()
    cfg.algo, cfg.max_inflight, cfg.max_tasks_per_launch = 7, 2, 16
    assert pico.pico_server_create(cfg)[0] == pico.PICO_EINVAL
    cfg.algo, cfg.max_inflight = pe, 0
    assert pico.pico_server_create(cfg)[0] == pico.PICO_EINVAL
    cfg.max_inflight, cfg.arena, cfg.arena_bytes = 2, 4096 + 8, 1 << 20  # misaligned arena
    assert pico.pico_server_create(cfg)[0] == pico.PICO_EINVAL
    cfg.arena = 4096
    cfg.max_large_slots = -1
    assert pico.pico_server_create(cfg)[0] == pico.PICO_EINVAL
    cfg.max_large_slots = 0
    cfg.class_bounds[0], cfg.class_bounds[1] = 5000, 100  # bounds out of order
    assert pico.pico_server_create(cfg)[0] == pico.PICO_EINVAL
    assert ctypes.sizeof(pico.ServerConfig) == 4 + 4 + 8 + 8 + 8 + 16 + 16 + 4 + 4
    assert pico.pico_server_destroy(None) == pico.PICO_OK


def test_schedule_argument_errors_need_no_device():
    """pico_coreness_schedule: algorithm and path checked before any device
    work; n == 0 records nothing and reports zero steps."""
    assert ctypes.sizeof(pico.PicoStep) == 64
    rc, count = pico.pico_coreness_schedule(None, None, 0, 0, pico.PICO_ALGO_HISTOCORE, None, None, 0, None,
                                            None, 0)
    assert (rc, count) == (pico.PICO_OK, 0)
    for bad in (pico.PICO_PATH_WG, pico.PICO_PO_STATIC, pico.PICO_ALGO_NBRCORE, 0x4000):
        rc, _ = pico.pico_coreness_schedule(None, None, 0, 0, bad, None, None, 0, None, None, 0)
        assert rc == pico.PICO_EINVAL, bad
    rc, _ = pico.pico_coreness_schedule(None, None, 0, 0, 0, None, None, 0, None, None, 4)
    assert rc == pico.PICO_EINVAL and "schedule" in pico.pico_last_error()
    rc, _ = pico.pico_coreness_schedule(None, None, 0, 0, 0, None, None, 0, None, None, -1)
    assert rc == pico.PICO_EINVAL


def test_batch_status_and_auto_sizes_need_no_device():
    """pico_batch_status checks its arguments before touching the device;
    PICO_ALGO_AUTO is accepted by the multi-graph size queries and sizes
    scratch and workspace for HistoCore (plus the per-graph choice)."""
    assert pico.pico_batch_status(None, 0, 0) == pico.PICO_OK
    assert pico.pico_batch_status(None, 0, -1) == pico.PICO_EINVAL
    assert pico.pico_batch_status(None, 0, 4) == pico.PICO_EINVAL
    a, h, p = pico.PICO_ALGO_AUTO, pico.PICO_ALGO_HISTOCORE, pico.PICO_ALGO_PEELONE
    assert pico.pico_task_scratch_bytes(1000, 9000, a) == pico.pico_task_scratch_bytes(1000, 9000, h)
    assert pico.pico_task_scratch_bytes(1000, 9000, p) < pico.pico_task_scratch_bytes(1000, 9000, h)
    assert pico.pico_batched_workspace_bytes(10, 1000, 9000, a) > pico.pico_batched_workspace_bytes(10, 1000, 9000, h)
    assert pico.pico_tasks_workspace_bytes(10) > 0
