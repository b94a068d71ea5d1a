"""HBM traffic of one kernel from two rocprofv3 counter runs.

rocprofv3 collects FETCH_SIZE and WRITE_SIZE (KiB per dispatch, the L2 <-> fabric
bytes) in two separate ``--pmc`` runs of the same command.  Both counters are
scaled by what they read for a plain copy kernel of known size (``bench.py
--pmc-copy`` runs ``torch.neg`` over 256 MiB before the workload), so the
reported bytes are in the same units as the copy's 256 MiB read and 256 MiB
written.  The summary records a hash of the library sources; ``bench.py``
reports the traffic only while the sources still hash to it.

Usage:
  python -m paper_0911_4498_amd.pmc_traffic FETCH_CSV WRITE_CSV KERNEL_SUBSTRING OUT_TXT \\
      --command "..." [--workload "..."] [--skip-idle]
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 256 * 1024 * 1024
COPY_KERNEL = "neg"


def source_hash() -> str:
    """sha256 over the library sources (kernels, headers, host driver)."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(HERE, "csrc", "*")) + glob.glob(os.path.join(HERE, "..", "include", "*.h")))
    for p in files:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def read_counter(path: str, counter: str) -> list[tuple[str, float]]:
    """(kernel name, value) per dispatch for one counter of a rocprofv3 counter CSV."""
    rows = []
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            name = r.get("Counter_Name", "")
            if name != counter:
                continue
            rows.append((r.get("Kernel_Name", ""), float(r.get("Counter_Value", "nan"))))
    if not rows:
        raise ValueError(f"{path}: no {counter} rows")
    return rows


def per_dispatch(rows, needle: str) -> list[float]:
    return [v for k, v in rows if needle in k]


def drop_idle(values: list[float]) -> list[float]:
    """Dispatches that moved under 1/1000 of the kernel's largest one: launches that returned
    at once (e.g. a gated second Gram-Schmidt pass that was not needed)."""
    top = max(values) if values else 0.0
    return [v for v in values if v >= 1e-3 * top]


def summarize(fetch_csv: str, write_csv: str, kernel: str, skip_idle: bool = False) -> dict:
    fr = read_counter(fetch_csv, "FETCH_SIZE")
    wr = read_counter(write_csv, "WRITE_SIZE")
    copy_f = [v for v in per_dispatch(fr, COPY_KERNEL) if v * 1024 > COPY_BYTES / 4]
    copy_w = [v for v in per_dispatch(wr, COPY_KERNEL) if v * 1024 > COPY_BYTES / 4]
    if not copy_f or not copy_w:
        raise ValueError("copy calibration dispatches not found (run bench.py with --pmc-copy)")
    f_fetch = COPY_BYTES / (statistics.median(copy_f) * 1024.0)
    f_write = COPY_BYTES / (statistics.median(copy_w) * 1024.0)
    kf = per_dispatch(fr, kernel)
    kw = per_dispatch(wr, kernel)
    if not kf or not kw:
        raise ValueError(f"kernel {kernel!r} not found in the counter files")
    n_all = len(kf)
    if skip_idle:
        kf, kw = drop_idle(kf), drop_idle(kw)
    fetch_b = statistics.mean(kf) * 1024.0 * f_fetch
    write_b = statistics.mean(kw) * 1024.0 * f_write
    return {
        "kernel": kernel,
        "dispatches_fetch": len(kf),
        "dispatches_write": len(kw),
        "idle_dispatches_skipped": n_all - len(kf),
        "fetch_kib_per_dispatch": statistics.mean(kf),
        "write_kib_per_dispatch": statistics.mean(kw),
        "copy_fetch_kib": statistics.median(copy_f),
        "copy_write_kib": statistics.median(copy_w),
        "copy_fetch_factor": f_fetch,
        "copy_write_factor": f_write,
        "fetch_bytes_per_launch": fetch_b,
        "write_bytes_per_launch": write_b,
        "traffic_bytes_per_launch": fetch_b + write_b,
        "source_sha256": source_hash(),
    }


def write_summary(out: str, s: dict, command: str, workload: str) -> None:
    with open(out, "w") as fh:
        fh.write(f"# HBM traffic of {s['kernel']} ({workload})\n")
        fh.write("# Two rocprofv3 counter runs of the same command (FETCH_SIZE, then WRITE_SIZE), each\n")
        fh.write("# scaled by the counter's reading for a 256 MiB copy (torch.neg) in the same run.\n")
        fh.write(f"# command: {command}\n")
        for key, val in s.items():
            fh.write(f"{key}: {val}\n")


def load_summary(path: str) -> dict | None:
    if not os.path.exists(path):
        return None
    out = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            v = v.strip()
            try:
                out[k.strip()] = float(v) if k.strip() not in ("kernel", "source_sha256") else v
            except ValueError:
                out[k.strip()] = v
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch_csv")
    ap.add_argument("write_csv")
    ap.add_argument("kernel")
    ap.add_argument("out")
    ap.add_argument("--command", default="")
    ap.add_argument("--workload", default="")
    ap.add_argument("--skip-idle", action="store_true", help="ignore dispatches that returned at once")
    a = ap.parse_args()
    s = summarize(a.fetch_csv, a.write_csv, a.kernel, a.skip_idle)
    write_summary(a.out, s, a.command, a.workload)
    for k, v in s.items():
        print(f"{k}: {v}")


if __name__ == "__main__":
    main()
