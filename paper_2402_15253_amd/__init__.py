"""Python binding of the gfx950 k-core library ``libpico.so``.

Argument marshalling only: every step of the decomposition runs in the HIP
kernels behind the C ABI declared in ``include/pico.h``.  PyTorch provides
device memory and streams.  There is no fallback: if the library has not been
built, every call raises.

Functions carry the C names (``pico_coreness``, ``pico_coreness_ws``,
``pico_workspace_bytes``, ``pico_validate_csr``, ``pico_status_string``,
``pico_last_error``, ``pico_version``); ``coreness`` is a convenience wrapper
that allocates the output (and optionally a workspace) with torch.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loaded first so the library binds to the HIP runtime torch uses

__all__ = [
    "PICO_OK", "PICO_EINVAL", "PICO_ENOMEM", "PICO_EHIP", "PICO_ENOTSUP", "PICO_EBADCSR",
    "PICO_ALGO_PEELONE", "PICO_ALGO_HISTOCORE", "PICO_OFFSETS_I64", "PICO_PATH_GRID", "PICO_PATH_WG",
    "PICO_PO_STATIC", "PICO_PO_ROLLBACK", "PICO_PO_GPP", "VARIANTS", "PICO_ALGO_CNTCORE", "PICO_ALGO_NBRCORE",
    "PATHS", "PicoError", "PicoStats",
    "pico_coreness", "pico_coreness_ws", "pico_coreness_update", "coreness_update",
    "pico_select_algorithm", "select_algorithm", "PICO_ALGO_AUTO", "SINGLE_ALGOS", "ALGO_NAMES",
    "pico_workspace_bytes", "pico_validate_csr",
    "pico_status_string", "pico_last_error", "pico_version", "coreness", "library_path",
    "load_library", "EXPORTED_SYMBOLS", "pico_profile_enable", "pico_profile_read",
    "pico_batched_workspace_bytes", "pico_coreness_batched", "coreness_batched", "BatchTune",
    "BatchStats", "largest_first", "Task", "ServerConfig", "Request", "Completion",
    "ServerStatus", "pico_task_scratch_bytes", "pico_tasks_workspace_bytes", "pico_coreness_tasks",
    "Server", "pico_server_create", "pico_server_submit", "pico_server_progress",
    "pico_server_query", "pico_server_destroy", "pico_probe_random_access", "probe_random_access",
    "PicoStep", "pico_coreness_schedule", "coreness_schedule", "pico_coreness_noalloc",
    "PICO_NOALLOC_SCRATCH_BYTES", "BATCH_ALGOS", "pico_batch_status", "batch_status",
]

PICO_OK, PICO_EINVAL, PICO_ENOMEM, PICO_EHIP, PICO_ENOTSUP, PICO_EBADCSR = 0, -1, -2, -3, -4, -5
PICO_ALGO_PEELONE, PICO_ALGO_HISTOCORE, PICO_ALGO_AUTO, PICO_OFFSETS_I64 = 0, 1, 2, 0x100
PICO_PATH_GRID, PICO_PATH_WG = 0x200, 0x400
PICO_PO_STATIC, PICO_PO_ROLLBACK, PICO_PO_GPP = 0x800, 0x1000, 0x2000
PICO_NOALLOC_SCRATCH_BYTES = 64 << 20  # static workspace of pico_coreness_noalloc
PATHS = {None: 0, "auto": 0, "grid": PICO_PATH_GRID, "wg": PICO_PATH_WG}
ALGOS = {"peelone": PICO_ALGO_PEELONE, "histocore": PICO_ALGO_HISTOCORE}
# batched, task-list and server calls may also choose per graph
BATCH_ALGOS = {**ALGOS, "auto": PICO_ALGO_AUTO}
# single-graph calls may also ask for the per-graph choice between the two
SINGLE_ALGOS = {**ALGOS, "auto": PICO_ALGO_AUTO}
ALGO_NAMES = {PICO_ALGO_PEELONE: "peelone", PICO_ALGO_HISTOCORE: "histocore"}
# PeelOne ablations (single-graph calls): no dynamic frontier; rollback decrement
PICO_ALGO_CNTCORE, PICO_ALGO_NBRCORE = 3, 4
VARIANTS = {"peelone-static": PICO_ALGO_PEELONE | PICO_PO_STATIC,
            "peelone-rollback": PICO_ALGO_PEELONE | PICO_PO_ROLLBACK,
            "gpp": PICO_ALGO_PEELONE | PICO_PO_GPP,
            # Index2core baselines (Table VI): every h-index rebuilt from the neighbours
            "cntcore": PICO_ALGO_CNTCORE, "nbrcore": PICO_ALGO_NBRCORE}

EXPORTED_SYMBOLS = ("pico_coreness", "pico_coreness_ws", "pico_coreness_update", "pico_select_algorithm",
                    "pico_workspace_bytes",
                    "pico_validate_csr", "pico_status_string", "pico_last_error", "pico_version",
                    "pico_profile_enable", "pico_profile_read", "pico_batched_workspace_bytes",
                    "pico_coreness_batched", "pico_task_scratch_bytes",
                    "pico_tasks_workspace_bytes", "pico_coreness_tasks", "pico_server_create",
                    "pico_server_submit", "pico_server_progress", "pico_server_query",
                    "pico_server_destroy", "pico_probe_random_access", "pico_coreness_schedule",
                    "pico_coreness_noalloc", "pico_batch_status")

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libpico.so")
_lib = None


class PicoError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        super().__init__(f"pico status {status}: {detail}")


class PicoStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("sub_rounds", ctypes.c_int64),
                ("scans", ctypes.c_int64), ("frontier_total", ctypes.c_int64),
                ("k_max", ctypes.c_int32), ("algo_used", ctypes.c_int32),
                ("elapsed_ms", ctypes.c_double), ("edges_scanned", ctypes.c_int64),
                ("atomics", ctypes.c_int64), ("buckets_scanned", ctypes.c_int64),
                ("pushes_dynamic", ctypes.c_int64), ("phase_ms", ctypes.c_double * 8)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "phase_ms"}
        d["phase_ms"] = [round(x, 4) for x in self.phase_ms]
        return d


class PicoStep(ctypes.Structure):
    """C ``pico_step``: one PeelOne level or HistoCore round (64 bytes)."""
    _fields_ = [(f, ctypes.c_int64) for f in ("key", "vertices", "work", "edges", "rounds", "ns",
                                               "scan_ns", "kind")]


STEP_FIELDS = tuple(f for f, _ in PicoStep._fields_)


class BatchTune(ctypes.Structure):
    _fields_ = [("lds_bytes", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("sum_wave_min", ctypes.c_int32), ("help_min_vertices", ctypes.c_int32)]

    def __init__(self, lds_bytes: int = -1, blocks_per_cu: int = 0, sum_wave_min: int = 0,
                 help_min_vertices: int = 0):
        super().__init__(lds_bytes, blocks_per_cu, sum_wave_min, help_min_vertices)

    def as_dict(self) -> dict:
        return {"lds_bytes": self.lds_bytes, "blocks_per_cu": self.blocks_per_cu,
                "sum_wave_min": self.sum_wave_min, "help_min_vertices": self.help_min_vertices}


class BatchStats(ctypes.Structure):
    _fields_ = [("graphs", ctypes.c_int64), ("iterations", ctypes.c_int64),
                ("atomics", ctypes.c_int64), ("frontier_total", ctypes.c_int64),
                ("edges_scanned", ctypes.c_int64), ("buckets_scanned", ctypes.c_int64),
                ("pushes", ctypes.c_int64), ("lds_graphs", ctypes.c_int64),
                ("workgroups", ctypes.c_int64), ("lds_bytes", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("helped_graphs", ctypes.c_int64),
                ("help_chunks", ctypes.c_int64), ("histocore_graphs", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class Task(ctypes.Structure):
    """C ``pico_task``: one graph of a task list."""
    _fields_ = [("offsets", ctypes.c_void_p), ("cols", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("m", ctypes.c_int64), ("out_core", ctypes.c_void_p), ("scratch", ctypes.c_void_p),
                ("scratch_bytes", ctypes.c_size_t)]


class ServerConfig(ctypes.Structure):
    """C ``pico_server_config``."""
    _fields_ = [("algo", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("max_tasks_per_launch", ctypes.c_int64), ("arena", ctypes.c_void_p),
                ("arena_bytes", ctypes.c_size_t), ("tune", BatchTune),
                ("class_bounds", ctypes.c_int64 * 2), ("max_large_slots", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Request(ctypes.Structure):
    """C ``pico_request``."""
    _fields_ = [("offsets", ctypes.c_void_p), ("cols", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("m", ctypes.c_int64), ("out_core", ctypes.c_void_p), ("tag", ctypes.c_int64)]


class Completion(ctypes.Structure):
    """C ``pico_completion``."""
    _fields_ = [("tag", ctypes.c_int64), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("t_submit_ns", ctypes.c_uint64), ("t_launch_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64)]


class ServerStatus(ctypes.Structure):
    """C ``pico_server_status``."""
    _fields_ = [(f, ctypes.c_int64) for f in ("waiting", "inflight", "ready", "busy_slots",
                                               "launches", "completed", "arena_used",
                                               "arena_bytes")]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libpico.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with paper_2402_15253_amd/build.py")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.pico_coreness.argtypes = [vp, vp, i64, i64, i32, vp, vp]
    lib.pico_coreness.restype = i32
    lib.pico_coreness_noalloc.argtypes = [vp, vp, i64, i64, i32, vp, vp]
    lib.pico_coreness_noalloc.restype = i32
    lib.pico_coreness_ws.argtypes = [vp, vp, i64, i64, i32, vp, vp, ctypes.c_size_t,
                                     ctypes.POINTER(PicoStats), vp]
    lib.pico_coreness_ws.restype = i32
    lib.pico_coreness_update.argtypes = [vp, vp, i64, i64, i32, vp, ctypes.c_int32, vp, vp,
                                         ctypes.c_size_t, ctypes.POINTER(PicoStats), vp]
    lib.pico_coreness_update.restype = i32
    lib.pico_coreness_schedule.argtypes = [vp, vp, i64, i64, i32, vp, vp, ctypes.c_size_t,
                                           ctypes.POINTER(PicoStats), vp, i64, ctypes.POINTER(ctypes.c_int64),
                                           vp]
    lib.pico_coreness_schedule.restype = i32
    lib.pico_select_algorithm.argtypes = [vp, vp, i64, i64, i32, vp, ctypes.c_size_t, ctypes.POINTER(i32),
                                          ctypes.POINTER(ctypes.c_int64), vp]
    lib.pico_select_algorithm.restype = i32
    lib.pico_workspace_bytes.argtypes = [i64, i64, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.pico_workspace_bytes.restype = i32
    lib.pico_validate_csr.argtypes = [vp, vp, i64, i64, i32, vp]
    lib.pico_validate_csr.restype = i32
    lib.pico_status_string.argtypes = [i32]
    lib.pico_status_string.restype = ctypes.c_char_p
    lib.pico_last_error.argtypes = []
    lib.pico_last_error.restype = ctypes.c_char_p
    lib.pico_version.argtypes = []
    lib.pico_version.restype = ctypes.c_char_p
    lib.pico_batched_workspace_bytes.argtypes = [i64, i64, i64, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.pico_batched_workspace_bytes.restype = i32
    lib.pico_coreness_batched.argtypes = [vp, vp, vp, i64, i64, i64, i32, vp, vp,
                                          ctypes.POINTER(BatchTune), vp, ctypes.c_size_t,
                                          ctypes.POINTER(BatchStats), vp]
    lib.pico_coreness_batched.restype = i32
    lib.pico_task_scratch_bytes.argtypes = [i64, i64, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.pico_task_scratch_bytes.restype = i32
    lib.pico_tasks_workspace_bytes.argtypes = [i64, ctypes.POINTER(ctypes.c_size_t)]
    lib.pico_tasks_workspace_bytes.restype = i32
    lib.pico_coreness_tasks.argtypes = [ctypes.POINTER(Task), i64, i32, ctypes.POINTER(BatchTune), vp,
                                        ctypes.c_size_t, ctypes.POINTER(BatchStats), vp]
    lib.pico_coreness_tasks.restype = i32
    lib.pico_batch_status.argtypes = [vp, ctypes.c_size_t, i64, vp, vp]
    lib.pico_batch_status.restype = i32
    lib.pico_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    lib.pico_server_create.restype = i32
    lib.pico_server_submit.argtypes = [vp, ctypes.POINTER(Request)]
    lib.pico_server_submit.restype = i32
    lib.pico_server_progress.argtypes = [vp, ctypes.POINTER(Completion), i32, ctypes.POINTER(i32)]
    lib.pico_server_progress.restype = i32
    lib.pico_server_query.argtypes = [vp, ctypes.POINTER(ServerStatus)]
    lib.pico_server_query.restype = i32
    lib.pico_server_destroy.argtypes = [vp]
    lib.pico_server_destroy.restype = i32
    lib.pico_probe_random_access.argtypes = [vp, ctypes.c_size_t, i64, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double), vp]
    lib.pico_probe_random_access.restype = i32
    lib.pico_profile_enable.argtypes = [i32]
    lib.pico_profile_enable.restype = i32
    lib.pico_profile_read.argtypes = [ctypes.POINTER(KernelStat), i32, ctypes.POINTER(i32)]
    lib.pico_profile_read.restype = i32
    _lib = lib
    return lib


def _ptr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return x.data_ptr() if x.numel() else None
    return int(x)


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def pico_status_string(status: int) -> str:
    return load_library().pico_status_string(status).decode()


def pico_last_error() -> str:
    return load_library().pico_last_error().decode()


def pico_version() -> str:
    return load_library().pico_version().decode()


def _check(rc: int) -> int:
    if rc != PICO_OK:
        raise PicoError(rc, f"{pico_status_string(rc)}: {pico_last_error()}")
    return rc


def pico_coreness(csr_offsets, csr_cols, n: int, m: int, algo: int, out_core, stream=None) -> int:
    """C ``pico_coreness``; returns the status code (does not raise)."""
    lib = load_library()
    return lib.pico_coreness(_ptr(csr_offsets), _ptr(csr_cols), n, m, algo, _ptr(out_core),
                             _stream(stream))


def pico_coreness_noalloc(csr_offsets, csr_cols, n: int, m: int, algo: int, out_core, stream=None) -> int:
    """C ``pico_coreness_noalloc``; returns the status code (does not raise)."""
    return load_library().pico_coreness_noalloc(_ptr(csr_offsets), _ptr(csr_cols), n, m, algo,
                                                _ptr(out_core), _stream(stream))


def pico_workspace_bytes(n: int, m: int, algo: int) -> int:
    """C ``pico_workspace_bytes``; raises PicoError on a bad status."""
    out = ctypes.c_size_t(0)
    _check(load_library().pico_workspace_bytes(n, m, algo, ctypes.byref(out)))
    return out.value


def pico_coreness_ws(csr_offsets, csr_cols, n: int, m: int, algo: int, out_core, workspace,
                     ws_bytes: int, stats: PicoStats | None = None, stream=None) -> int:
    """C ``pico_coreness_ws``; returns the status code (does not raise)."""
    lib = load_library()
    return lib.pico_coreness_ws(_ptr(csr_offsets), _ptr(csr_cols), n, m, algo, _ptr(out_core),
                                _ptr(workspace), ws_bytes,
                                ctypes.byref(stats) if stats is not None else None,
                                _stream(stream))


def pico_coreness_schedule(csr_offsets, csr_cols, n: int, m: int, algo: int, out_core, workspace,
                           ws_bytes: int, stats: PicoStats | None, steps, cap: int, stream=None):
    """C ``pico_coreness_schedule`` (``steps``: device buffer of cap * 64
    bytes); returns (status, number of steps the run took)."""
    count = ctypes.c_int64(0)
    rc = load_library().pico_coreness_schedule(_ptr(csr_offsets), _ptr(csr_cols), n, m, algo, _ptr(out_core),
                                               _ptr(workspace), ws_bytes,
                                               ctypes.byref(stats) if stats is not None else None,
                                               _ptr(steps), cap, ctypes.byref(count), _stream(stream))
    return rc, count.value


def coreness_schedule(offsets: torch.Tensor, cols: torch.Tensor, algo="peelone", *, cap: int = 1 << 16,
                      workspace=None, stream=None):
    """Coreness plus the run's schedule on the grid path: (core, stats,
    steps), steps an int64 tensor on the host of shape [count, 8] whose
    columns are STEP_FIELDS (PeelOne: one row per non-empty level; HistoCore:
    one row per round).  Raises PicoError if the run took more than ``cap``
    steps."""
    if cols.dtype != torch.int32:
        raise TypeError("cols must be int32")
    n = offsets.numel() - 1
    m = cols.numel()
    a = algo_code(algo, offsets)
    out = torch.empty(max(n, 0), dtype=torch.int32, device=offsets.device)
    if workspace is None:
        workspace = workspace_for(n, m, a, offsets.device)
    steps = torch.zeros((max(cap, 1), len(STEP_FIELDS)), dtype=torch.int64, device=offsets.device)
    st = PicoStats()
    rc, count = pico_coreness_schedule(offsets, cols, n, m, a, out, workspace, workspace.numel(), st, steps,
                                       cap, stream)
    _check(rc)
    if count > cap:
        raise PicoError(PICO_ENOMEM, f"schedule of {count} steps does not fit cap {cap}")
    return out, st.as_dict(), steps[:count].cpu()


def pico_profile_enable(on: bool) -> int:
    """C ``pico_profile_enable`` (per host thread)."""
    return load_library().pico_profile_enable(1 if on else 0)


def pico_profile_read() -> dict:
    """C ``pico_profile_read``: {kernel name: (launches, total_ms)}."""
    lib = load_library()
    count = ctypes.c_int(0)
    _check(lib.pico_profile_read(None, 0, ctypes.byref(count)))
    arr = (KernelStat * max(count.value, 1))()
    _check(lib.pico_profile_read(arr, count.value, ctypes.byref(count)))
    return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(count.value)}


def pico_batched_workspace_bytes(num_graphs: int, total_n: int, total_m: int, algo: int) -> int:
    """C ``pico_batched_workspace_bytes``; raises PicoError on a bad status."""
    out = ctypes.c_size_t(0)
    _check(load_library().pico_batched_workspace_bytes(num_graphs, total_n, total_m, algo,
                                                       ctypes.byref(out)))
    return out.value


def pico_task_scratch_bytes(n: int, m: int, algo: int) -> int:
    """C ``pico_task_scratch_bytes``; raises PicoError on a bad status."""
    out = ctypes.c_size_t(0)
    _check(load_library().pico_task_scratch_bytes(n, m, algo, ctypes.byref(out)))
    return out.value


def pico_tasks_workspace_bytes(num_tasks: int) -> int:
    """C ``pico_tasks_workspace_bytes``; raises PicoError on a bad status."""
    out = ctypes.c_size_t(0)
    _check(load_library().pico_tasks_workspace_bytes(num_tasks, ctypes.byref(out)))
    return out.value


def pico_coreness_tasks(tasks, algo: int, tune: BatchTune | None, workspace, ws_bytes: int,
                        stats: BatchStats | None = None, stream=None) -> int:
    """C ``pico_coreness_tasks`` over a sequence of Task; returns the status code."""
    arr = (Task * max(len(tasks), 1))(*tasks)
    return load_library().pico_coreness_tasks(arr, len(tasks), algo,
                                              ctypes.byref(tune) if tune is not None else None,
                                              _ptr(workspace), ws_bytes,
                                              ctypes.byref(stats) if stats is not None else None,
                                              _stream(stream))


def pico_coreness_batched(graph_vptr, csr_offsets, csr_cols, num_graphs: int, total_n: int,
                          total_m: int, algo: int, order, out_core, tune: BatchTune | None,
                          workspace, ws_bytes: int, stats: BatchStats | None = None,
                          stream=None) -> int:
    """C ``pico_coreness_batched``; returns the status code (does not raise)."""
    lib = load_library()
    return lib.pico_coreness_batched(_ptr(graph_vptr), _ptr(csr_offsets), _ptr(csr_cols),
                                     num_graphs, total_n, total_m, algo, _ptr(order),
                                     _ptr(out_core), ctypes.byref(tune) if tune is not None else None,
                                     _ptr(workspace), ws_bytes,
                                     ctypes.byref(stats) if stats is not None else None,
                                     _stream(stream))


def pico_batch_status(workspace, ws_bytes: int, count: int, status=None, stream=None) -> int:
    """C ``pico_batch_status`` (``status``: host int32 numpy array of ``count``
    entries, or None); returns the status code."""
    ptr = status.ctypes.data if status is not None else None
    return load_library().pico_batch_status(_ptr(workspace), ws_bytes, count, ptr, _stream(stream))


def batch_status(workspace, count: int, stream=None):
    """(summary status, int32 numpy array of per-graph status words) of the
    last batched or task-list call on ``workspace``."""
    import numpy as np
    out = np.zeros(max(count, 0), dtype=np.int32)
    rc = pico_batch_status(workspace, workspace.numel(), count, out if count else None, stream)
    return rc, out


def largest_first(vptr: torch.Tensor) -> torch.Tensor:
    """Processing order for a batch: graphs by decreasing vertex count."""
    sizes = vptr[1:] - vptr[:-1]
    return torch.argsort(sizes, descending=True, stable=True).to(torch.int32)


def coreness_batched(batch, algo="peelone", *, order="largest_first", tune=None, out=None,
                     workspace=None, with_stats: bool = False, stream=None):
    """Coreness of every vertex of a device-resident packed batch (object with
    vptr, offsets, cols tensors).  Raises PicoError on failure; waits for the
    result when with_stats is set, otherwise returns once enqueued."""
    a = BATCH_ALGOS[algo] if isinstance(algo, str) else int(algo)
    G = batch.vptr.numel() - 1
    total_n = batch.offsets.numel() - 1
    total_m = batch.cols.numel()
    if isinstance(order, str):
        order = largest_first(batch.vptr)
    if out is None:
        out = torch.empty(max(total_n, 0), dtype=torch.int32, device=batch.offsets.device)
    if workspace is None:
        nbytes = pico_batched_workspace_bytes(G, total_n, total_m, a)
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=batch.offsets.device)
    st = BatchStats() if with_stats else None
    _check(pico_coreness_batched(batch.vptr, batch.offsets, batch.cols, G, total_n, total_m, a, order,
                                 out, tune, workspace, workspace.numel(), st, stream=stream))
    return (out, st.as_dict()) if with_stats else out


def pico_validate_csr(csr_offsets, csr_cols, n: int, m: int, algo: int, stream=None) -> int:
    """C ``pico_validate_csr``; returns the status code."""
    return load_library().pico_validate_csr(_ptr(csr_offsets), _ptr(csr_cols), n, m, algo,
                                            _stream(stream))


def algo_code(algo, offsets: torch.Tensor, path=None) -> int:
    """The C algo word: algorithm, offset width and path ("grid", "wg" or
    None/"auto" for the library's choice by size)."""
    if isinstance(algo, str):
        a = VARIANTS[algo] if algo in VARIANTS else SINGLE_ALGOS[algo]
    else:
        a = int(algo)
    a |= PATHS[path]
    if offsets.dtype == torch.int64:
        a |= PICO_OFFSETS_I64
    elif offsets.dtype != torch.int32:
        raise TypeError("offsets must be int32 or int64")
    return a


def workspace_for(n: int, m: int, algo: int, device) -> torch.Tensor:
    """A torch-allocated device workspace of pico_workspace_bytes(n, m, algo)."""
    nbytes = pico_workspace_bytes(n, m, algo)
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def coreness(offsets: torch.Tensor, cols: torch.Tensor, algo="peelone", *, out=None,
             workspace=None, with_stats: bool = False, stream=None, path=None):
    """Coreness of every vertex of a device-resident CSR graph (int32 tensor).

    ``offsets``: int32/int64 [n+1] on the GPU; ``cols``: int32 [m] on the GPU.
    ``path``: None (by size), "grid" (persistent kernels) or "wg" (one
    workgroup, values in LDS).  Raises PicoError on failure.  With
    ``with_stats`` returns (core, stats).
    """
    if cols.dtype != torch.int32:
        raise TypeError("cols must be int32")
    n = offsets.numel() - 1
    m = cols.numel()
    a = algo_code(algo, offsets, path)
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=offsets.device)
    if workspace is None:
        workspace = workspace_for(n, m, a, offsets.device)
    st = PicoStats()
    _check(pico_coreness_ws(offsets, cols, n, m, a, out, workspace, workspace.numel(), st,
                            stream=stream))
    return (out, st.as_dict()) if with_stats else out


def pico_select_algorithm(csr_offsets, csr_cols, n: int, m: int, algo: int, workspace, ws_bytes: int,
                          stream=None):
    """C ``pico_select_algorithm``: returns (status, chosen algo code, [H, sampled, in_frontier])."""
    out = ctypes.c_int(0)
    feat = (ctypes.c_int64 * 3)()
    rc = load_library().pico_select_algorithm(_ptr(csr_offsets), _ptr(csr_cols), n, m, algo, _ptr(workspace),
                                              ws_bytes, ctypes.byref(out), feat, _stream(stream))
    return rc, out.value, list(feat)


def select_algorithm(offsets: torch.Tensor, cols: torch.Tensor, workspace=None, stream=None):
    """The algorithm PICO_ALGO_AUTO runs on this graph: (name, features
    {"h_index", "sampled", "in_first_frontier"})."""
    n = offsets.numel() - 1
    m = cols.numel()
    a = algo_code("auto", offsets)
    if workspace is None:
        workspace = workspace_for(n, m, a, offsets.device)
    rc, chosen, f = pico_select_algorithm(offsets, cols, n, m, a, workspace, workspace.numel(), stream)
    _check(rc)
    return ALGO_NAMES[chosen], {"h_index": f[0], "sampled": f[1], "in_first_frontier": f[2]}


def pico_probe_random_access(buf, nbytes: int, ops: int, stream=None):
    """C ``pico_probe_random_access``: (status, gathers/s, atomics/s)."""
    g, a = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = load_library().pico_probe_random_access(_ptr(buf), nbytes, ops, ctypes.byref(g), ctypes.byref(a),
                                                 _stream(stream))
    return rc, g.value, a.value


def probe_random_access(nbytes: int, ops: int = 1 << 28, device="cuda", stream=None) -> dict:
    """Random 4-byte gathers and atomic adds per second over a scratch array
    of ``nbytes`` bytes on ``device`` (allocated here and freed on return)."""
    words = max(1, int(nbytes) // 4)
    buf = torch.zeros(words, dtype=torch.int32, device=device)
    rc, g, a = pico_probe_random_access(buf, words * 4, int(ops), stream)
    _check(rc)
    del buf
    return {"bytes": words * 4, "ops": int(ops), "gathers_per_s": g, "atomics_per_s": a}


def pico_coreness_update(csr_offsets, csr_cols, n: int, m: int, algo: int, prev_core, bound_add: int,
                         out_core, workspace, ws_bytes: int, stats: PicoStats | None = None,
                         stream=None) -> int:
    """C ``pico_coreness_update``; returns the status code."""
    return load_library().pico_coreness_update(_ptr(csr_offsets), _ptr(csr_cols), n, m, algo,
                                               _ptr(prev_core), bound_add, _ptr(out_core),
                                               _ptr(workspace), ws_bytes,
                                               ctypes.byref(stats) if stats is not None else None,
                                               _stream(stream))


def coreness_update(offsets: torch.Tensor, cols: torch.Tensor, prev_core: torch.Tensor,
                    bound_add: int = 0, *, out=None, workspace=None, with_stats: bool = False,
                    stream=None, path=None):
    """Coreness of a changed graph from upper bounds ``prev_core + bound_add``
    (HistoCore started from them): after edge deletions the old coreness with
    bound_add 0, after b insertions the old coreness with bound_add b.
    ``out`` may be ``prev_core`` (in-place update)."""
    if cols.dtype != torch.int32 or prev_core.dtype != torch.int32:
        raise TypeError("cols and prev_core must be int32")
    n = offsets.numel() - 1
    m = cols.numel()
    if prev_core.numel() != max(n, 0):
        raise ValueError("prev_core must hold one value per vertex")
    a = algo_code("histocore", offsets, path)
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=offsets.device)
    if workspace is None:
        workspace = workspace_for(n, m, a, offsets.device)
    st = PicoStats()
    _check(pico_coreness_update(offsets, cols, n, m, a, prev_core, bound_add, out, workspace,
                                workspace.numel(), st, stream=stream))
    return (out, st.as_dict()) if with_stats else out


def pico_server_create(cfg: ServerConfig):
    """C ``pico_server_create``: returns (status, handle)."""
    h = ctypes.c_void_p(0)
    rc = load_library().pico_server_create(ctypes.byref(cfg), ctypes.byref(h))
    return rc, h


def pico_server_submit(handle, req: Request) -> int:
    """C ``pico_server_submit``; returns the status code."""
    return load_library().pico_server_submit(handle, ctypes.byref(req))


def pico_server_progress(handle, done, max_done: int):
    """C ``pico_server_progress`` into a ctypes array of Completion: returns
    (status, number of completions written)."""
    nd = ctypes.c_int(0)
    rc = load_library().pico_server_progress(handle, done, max_done, ctypes.byref(nd))
    return rc, nd.value


def pico_server_query(handle):
    """C ``pico_server_query``: returns (status, ServerStatus)."""
    st = ServerStatus()
    rc = load_library().pico_server_query(handle, ctypes.byref(st))
    return rc, st


def pico_server_destroy(handle) -> int:
    """C ``pico_server_destroy``; returns the status code."""
    return load_library().pico_server_destroy(handle)


class Server:
    """The C request server (``pico_server_*``) over a torch-allocated arena.

    ``submit`` queues a request for a device-resident graph (int64 offsets)
    and a device output; ``progress`` reaps, launches and returns completions
    as a list of Completion.  ``close`` waits for launches in flight."""

    def __init__(self, algo="peelone", *, arena_bytes: int, max_inflight: int = 4,
                 max_tasks_per_launch: int = 4096, tune: BatchTune | None = None,
                 class_bounds=(0, 0), max_large_slots: int = 0, device=None):
        lib = load_library()
        self._arena = torch.empty(max(arena_bytes, 256), dtype=torch.uint8, device=device or "cuda")
        cfg = ServerConfig()
        cfg.algo = BATCH_ALGOS[algo] if isinstance(algo, str) else int(algo)
        cfg.max_inflight = max_inflight
        cfg.max_tasks_per_launch = max_tasks_per_launch
        cfg.arena = self._arena.data_ptr()
        cfg.arena_bytes = arena_bytes
        cfg.tune = tune if tune is not None else BatchTune()
        cfg.class_bounds[0], cfg.class_bounds[1] = class_bounds
        cfg.max_large_slots = max_large_slots
        h = ctypes.c_void_p(0)
        torch.cuda.synchronize()
        _check(lib.pico_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._lib = lib
        self._buf = (Completion * 4096)()
        self._nd = ctypes.c_int(0)
        self._req = Request()

    def submit(self, offsets, cols, n: int, m: int, out_core, tag: int) -> None:
        r = self._req
        r.offsets, r.cols, r.n, r.m = _ptr(offsets), _ptr(cols), n, m
        r.out_core, r.tag = _ptr(out_core), tag
        _check(self._lib.pico_server_submit(self._h, ctypes.byref(r)))

    def submit_ptrs(self, offsets: int, cols: int, n: int, m: int, out_core: int, tag: int) -> None:
        r = self._req
        r.offsets, r.cols, r.n, r.m, r.out_core, r.tag = offsets, cols, n, m, out_core, tag
        _check(self._lib.pico_server_submit(self._h, ctypes.byref(r)))

    def progress(self) -> list:
        _check(self._lib.pico_server_progress(self._h, self._buf, len(self._buf),
                                              ctypes.byref(self._nd)))
        return [self._buf[i] for i in range(self._nd.value)]

    def progress_raw(self):
        """(count, buffer): completions stay in the shared buffer until the next call."""
        _check(self._lib.pico_server_progress(self._h, self._buf, len(self._buf),
                                              ctypes.byref(self._nd)))
        return self._nd.value, self._buf

    def status(self) -> dict:
        st = ServerStatus()
        _check(self._lib.pico_server_query(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self) -> None:
        if self._h is not None and self._h.value:
            _check(self._lib.pico_server_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
