"""Summaries of rocprofv3 runs of bench.py (kernel time and HBM traffic).

Usage (each run writes CSV files under its -d directory):

  rocprofv3 --kernel-trace --stats --output-format csv -d DIR -o run -- \\
      python3 bench.py ...                       # kernel durations
  rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR_F -o run -- \\
      python3 bench.py ... --copy-calibration    # bytes read per dispatch (KiB)
  rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR_W -o run -- \\
      python3 bench.py ... --copy-calibration    # bytes written per dispatch (KiB)

  python -m paper_2402_15253_amd.profiling stats DIR
  python -m paper_2402_15253_amd.profiling traffic DIR_F DIR_W

The traffic summary scales each counter by what the same counter reads for
the plain device-to-device copy that bench.py's --copy-calibration performs
(a known number of bytes read and written), and reports per-launch bytes for
the decomposition kernels.  It also records a hash of the HIP sources, so a
reader can tell whether the kernels changed since the counters were taken.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNELS = ("po_persistent", "hc_persistent")
COPY_MARK = "copy"  # torch's copy kernel names contain this


def source_hash() -> str:
    """Hash of the HIP sources and header the kernels are built from."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(HERE, "csrc", "*"))) + \
        [os.path.join(HERE, "..", "include", "pico.h")]
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def _find(d: str, suffix: str) -> str:
    hits = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def kernel_stats(d: str) -> dict:
    """{kernel short name: (calls, avg_ms, total_ms)} from a --stats run."""
    out = {}
    with open(_find(d, "kernel_stats.csv")) as f:
        for row in csv.DictReader(f):
            name = row["Name"]
            for k in KERNELS:
                if k in name:
                    out[k] = (int(row["Calls"]), float(row["AverageNs"]) / 1e6,
                              float(row["TotalDurationNs"]) / 1e6)
    return out


def _counter_rows(d: str, counter: str):
    path = _find(d, "counter_collection.csv")
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") == counter:
                yield row["Kernel_Name"], float(row["Counter_Value"])


def counter_per_dispatch(d: str, counter: str) -> dict:
    """Mean counter value per dispatch, by kernel short name ('copy' for the
    calibration copy, which is the largest copy dispatch of the run)."""
    acc, copy_max = {}, 0.0
    for name, val in _counter_rows(d, counter):
        for k in KERNELS:
            if k in name:
                s, c = acc.get(k, (0.0, 0))
                acc[k] = (s + val, c + 1)
        if COPY_MARK in name.lower() or "elementwise" in name:
            copy_max = max(copy_max, val)
    out = {k: s / c for k, (s, c) in acc.items()}
    out["copy"] = copy_max
    return out


def traffic(dir_fetch: str, dir_write: str, copy_bytes: int) -> dict:
    """Per-launch HBM bytes read and written, scaled by the copy calibration."""
    fetch = counter_per_dispatch(dir_fetch, "FETCH_SIZE")
    write = counter_per_dispatch(dir_write, "WRITE_SIZE")
    f_scale = copy_bytes / fetch["copy"] if fetch.get("copy") else None
    w_scale = copy_bytes / write["copy"] if write.get("copy") else None
    out = {"copy_bytes": copy_bytes, "fetch_factor": f_scale, "write_factor": w_scale}
    for k in KERNELS:
        if k in fetch and k in write and f_scale and w_scale:
            rd = fetch[k] * f_scale
            wr = write[k] * w_scale
            out[k] = {"read_bytes": int(rd), "write_bytes": int(wr), "bytes": int(rd + wr),
                      "fetch_kib_raw": fetch[k], "write_kib_raw": write[k]}
    return out


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        st = kernel_stats(argv[1])
        print(f"source_hash: {source_hash()}")
        for k, (calls, avg, tot) in st.items():
            print(f"{k}: calls {calls} avg_ms {avg:.4f} total_ms {tot:.3f}")
        return 0
    if len(argv) >= 3 and argv[0] == "traffic":
        copy_bytes = int(argv[3]) if len(argv) > 3 else 1 << 30
        t = traffic(argv[1], argv[2], copy_bytes)
        print(f"source_hash: {source_hash()}")
        for k, v in t.items():
            print(f"{k}: {v}")
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
