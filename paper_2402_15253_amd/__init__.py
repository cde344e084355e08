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
    "PICO_ALGO_PEELONE", "PICO_ALGO_HISTOCORE", "PICO_OFFSETS_I64", "PicoError", "PicoStats",
    "pico_coreness", "pico_coreness_ws", "pico_workspace_bytes", "pico_validate_csr",
    "pico_status_string", "pico_last_error", "pico_version", "coreness", "library_path",
    "load_library", "EXPORTED_SYMBOLS", "pico_profile_enable", "pico_profile_read",
]

PICO_OK, PICO_EINVAL, PICO_ENOMEM, PICO_EHIP, PICO_ENOTSUP, PICO_EBADCSR = 0, -1, -2, -3, -4, -5
PICO_ALGO_PEELONE, PICO_ALGO_HISTOCORE, PICO_OFFSETS_I64 = 0, 1, 0x100
ALGOS = {"peelone": PICO_ALGO_PEELONE, "histocore": PICO_ALGO_HISTOCORE}

EXPORTED_SYMBOLS = ("pico_coreness", "pico_coreness_ws", "pico_workspace_bytes",
                    "pico_validate_csr", "pico_status_string", "pico_last_error", "pico_version",
                    "pico_profile_enable", "pico_profile_read")

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
                ("k_max", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("elapsed_ms", ctypes.c_double), ("edges_scanned", ctypes.c_int64),
                ("atomics", ctypes.c_int64), ("buckets_scanned", ctypes.c_int64),
                ("pushes_dynamic", ctypes.c_int64), ("phase_ms", ctypes.c_double * 8)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("reserved", "phase_ms")}
        d["phase_ms"] = [round(x, 4) for x in self.phase_ms]
        return d


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
    lib.pico_coreness_ws.argtypes = [vp, vp, i64, i64, i32, vp, vp, ctypes.c_size_t,
                                     ctypes.POINTER(PicoStats), vp]
    lib.pico_coreness_ws.restype = i32
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


def pico_validate_csr(csr_offsets, csr_cols, n: int, m: int, algo: int, stream=None) -> int:
    """C ``pico_validate_csr``; returns the status code."""
    return load_library().pico_validate_csr(_ptr(csr_offsets), _ptr(csr_cols), n, m, algo,
                                            _stream(stream))


def algo_code(algo, offsets: torch.Tensor) -> int:
    a = ALGOS[algo] if isinstance(algo, str) else int(algo)
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
             workspace=None, with_stats: bool = False, stream=None):
    """Coreness of every vertex of a device-resident CSR graph (int32 tensor).

    ``offsets``: int32/int64 [n+1] on the GPU; ``cols``: int32 [m] on the GPU.
    Raises PicoError on failure.  With ``with_stats`` returns (core, stats).
    """
    if cols.dtype != torch.int32:
        raise TypeError("cols must be int32")
    n = offsets.numel() - 1
    m = cols.numel()
    a = algo_code(algo, offsets)
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.int32, device=offsets.device)
    if workspace is None:
        workspace = workspace_for(n, m, a, offsets.device)
    st = PicoStats()
    _check(pico_coreness_ws(offsets, cols, n, m, a, out, workspace, workspace.numel(), st,
                            stream=stream))
    return (out, st.as_dict()) if with_stats else out
