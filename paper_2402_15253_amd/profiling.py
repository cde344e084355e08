"""Summaries of rocprofv3 runs of bench.py (kernel time and HBM traffic).

Usage (each run writes CSV files under its -d directory):

  rocprofv3 --kernel-trace --stats --output-format csv -d DIR -o run -- \\
      python3 bench.py ...                       # kernel durations
  rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR_F -o run -- \\
      python3 bench.py ... --copy-calibration    # bytes read per dispatch (KiB)
  rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR_W -o run -- \\
      python3 bench.py ... --copy-calibration    # bytes written per dispatch (KiB)

  python -m paper_2402_15253_amd.profiling stats DIR
  python -m paper_2402_15253_amd.profiling traffic DIR_F DIR_W CONFIG
  python -m paper_2402_15253_amd.profiling counters DIR   # any --pmc run

The traffic summary scales each counter by what the same counter reads for
the 1 GiB device-to-device copy that bench.py's --copy-calibration performs
(2^30 bytes read and 2^30 written), and reports per-launch bytes for the
decomposition kernels.  Each kernel's line carries a hash of the sources it is
built from; bench.py uses a traffic figure only while that hash still matches.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
KERNEL_SOURCES = {
    "po_persistent": ("peelone.hip", "common.hpp"),
    "hc_persistent": ("histocore.hip", "common.hpp"),
    "batched_kernel": ("batched.hip", "common.hpp"),
    "po_small": ("batched.hip", "common.hpp"),
    "hc_small": ("batched.hip", "common.hpp"),
}
KERNELS = tuple(KERNEL_SOURCES)
COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 1 << 30


_COMMENT = re.compile(r"//[^\n]*|/\*.*?\*/", re.S)


def code_hash(sources) -> str:
    """Hash of (file name, text) pairs with comments and whitespace removed, so
    an edit of the comments alone keeps the hash while any change to the code
    changes it."""
    h = hashlib.sha256()
    for name, text in sources:
        h.update(name.encode())
        h.update("".join(_COMMENT.sub(" ", text).split()).encode())
    return h.hexdigest()[:16]


def source_hash(kernel: str) -> str:
    """Hash of the HIP code one kernel is built from (see code_hash)."""
    texts = []
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(HERE, "csrc", name), encoding="utf-8") as f:
            texts.append((name, f.read()))
    return code_hash(texts)


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def kernel_stats(d: str) -> dict:
    """{kernel short name: (calls, avg_ms, total_ms)} from a --stats run."""
    out = {}
    with open(_find(d, "kernel_stats.csv")) as f:
        for row in csv.DictReader(f):
            for k in KERNELS:
                if k in row["Name"]:
                    out[k] = (int(row["Calls"]), float(row["AverageNs"]) / 1e6,
                              float(row["TotalDurationNs"]) / 1e6)
    return out


def counter_per_dispatch(d: str, counter: str) -> dict:
    """Mean counter value (KiB) per dispatch of each decomposition kernel, and
    the calibration copy's value ('copy'): the last copyBuffer dispatch of at
    least a quarter of the largest copy's value.  bench.py's
    --copy-calibration copy runs after everything it measures; input
    generation may dispatch larger copies before it, and small copies may
    follow it."""
    acc, copies = {}, []
    with open(_find(d, "counter_collection.csv")) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            name, val = row["Kernel_Name"], float(row["Counter_Value"])
            for k in KERNELS:
                if k in name:
                    s, c = acc.get(k, (0.0, 0))
                    acc[k] = (s + val, c + 1)
            if COPY_KERNEL in name:
                copies.append((int(row.get("Dispatch_Id") or 0), val))
    out = {k: s / c for k, (s, c) in acc.items()}
    big = max((v for _, v in copies), default=0.0)
    out["copy"] = max((c for c in copies if c[1] >= 0.25 * big), default=(0, 0.0))[1]
    return out


def traffic(dir_fetch: str, dir_write: str) -> dict:
    """Per-launch HBM bytes read and written, scaled by the copy calibration."""
    fetch = counter_per_dispatch(dir_fetch, "FETCH_SIZE")
    write = counter_per_dispatch(dir_write, "WRITE_SIZE")
    f_scale = COPY_BYTES / fetch["copy"] if fetch.get("copy") else None
    w_scale = COPY_BYTES / write["copy"] if write.get("copy") else None
    out = {"fetch_factor": f_scale, "write_factor": w_scale,
           "copy_fetch_kib": fetch.get("copy"), "copy_write_kib": write.get("copy")}
    for k in KERNELS:
        if k in fetch and k in write and f_scale and w_scale:
            rd, wr = fetch[k] * f_scale, write[k] * w_scale
            out[k] = {"read_bytes": int(rd), "write_bytes": int(wr), "bytes": int(rd + wr),
                      "fetch_kib_raw": round(fetch[k], 1), "write_kib_raw": round(write[k], 1)}
    return out


_LINE = re.compile(r"^traffic (\w+) ([\w-]+) bytes_per_launch=(\d+) source=([0-9a-f]+)\s*$")


def format_traffic(t: dict, config: str) -> str:
    lines = [f"fetch_factor {t['fetch_factor']:.4f} (copy of 2^30 B read as "
             f"{t['copy_fetch_kib']:.1f} KiB FETCH_SIZE)",
             f"write_factor {t['write_factor']:.4f} (copy of 2^30 B written as "
             f"{t['copy_write_kib']:.1f} KiB WRITE_SIZE)"]
    for k in KERNELS:
        if k in t:
            v = t[k]
            lines.append(f"{k}: read {v['read_bytes']} B, write {v['write_bytes']} B per launch "
                         f"(raw FETCH_SIZE {v['fetch_kib_raw']} KiB, WRITE_SIZE {v['write_kib_raw']} KiB)")
            lines.append(f"traffic {k} {config} bytes_per_launch={v['bytes']} source={source_hash(k)}")
    return "\n".join(lines)


def recorded_traffic(kernel: str, config: str) -> int | None:
    """HBM bytes per launch of `kernel` on `config` from the committed
    summaries under profiles/, if the kernel's sources are unchanged since."""
    want = source_hash(kernel)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")) +
                       glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        with open(path) as f:
            for line in f:
                m = _LINE.match(line.strip())
                if m and m.group(1) == kernel and m.group(2) == config and m.group(4) == want:
                    return int(m.group(3))
    return None


def counters(d: str) -> dict:
    """{kernel short name: {counter: mean value per dispatch}} of a --pmc run
    (every counter the run collected, decomposition kernels only)."""
    acc = {}
    with open(_find(d, "counter_collection.csv")) as f:
        for row in csv.DictReader(f):
            for k in KERNELS:
                if k in row["Kernel_Name"]:
                    key = (k, row["Counter_Name"])
                    s, c = acc.get(key, (0.0, 0))
                    acc[key] = (s + float(row["Counter_Value"]), c + 1)
    out = {}
    for (k, name), (s, c) in acc.items():
        out.setdefault(k, {})[name] = s / c
    return out


def format_counters(c: dict, cus: int = 256) -> str:
    """One line per kernel and counter, plus the derived figures the
    collected counters allow: occupancy (SQ_WAVE_CYCLES over GRBM_GUI_ACTIVE,
    as rocprofv3's OccupancyPercent with 32 wave slots per CU), LDS bank
    conflicts per LDS access cycle, L2 hit rate, and atomic requests."""
    lines = []
    for k in sorted(c):
        v = c[k]
        for name in sorted(v):
            lines.append(f"{k}: {name} {v[name]:.6g} source={source_hash(k)}")
        if "SQ_WAVE_CYCLES" in v and v.get("GRBM_GUI_ACTIVE"):
            occ = 400.0 * v["SQ_WAVE_CYCLES"] / v["GRBM_GUI_ACTIVE"] / cus / 32
            lines.append(f"{k}: derived occupancy_percent {occ:.2f}")
        if "SQ_LDS_BANK_CONFLICT" in v and v.get("SQ_LDS_IDX_ACTIVE"):
            busy = v["SQ_LDS_IDX_ACTIVE"] - v["SQ_LDS_BANK_CONFLICT"]
            if busy > 0:
                lines.append(f"{k}: derived lds_bank_conflicts_per_access {v['SQ_LDS_BANK_CONFLICT'] / busy:.4f}")
        if "TCC_HIT_sum" in v and "TCC_MISS_sum" in v and v["TCC_HIT_sum"] + v["TCC_MISS_sum"] > 0:
            hit = v["TCC_HIT_sum"] / (v["TCC_HIT_sum"] + v["TCC_MISS_sum"])
            lines.append(f"{k}: derived l2_hit_rate {hit:.4f}")
    return "\n".join(lines)


def main(argv):
    if len(argv) >= 2 and argv[0] == "counters":
        print(format_counters(counters(argv[1])))
        return 0
    if len(argv) >= 2 and argv[0] == "stats":
        for k, (calls, avg, tot) in kernel_stats(argv[1]).items():
            print(f"{k}: calls {calls} avg_ms {avg:.4f} total_ms {tot:.3f} source={source_hash(k)}")
        return 0
    if len(argv) >= 4 and argv[0] == "traffic":
        print(format_traffic(traffic(argv[1], argv[2]), argv[3]))
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
