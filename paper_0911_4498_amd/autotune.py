"""Measured FFT schedules for the single-series products, cached per (N, L).

``ssa_tune_fft`` times the candidate schedules of a product (transform length M' = M/2,
its split M1 x M2, the columns per workgroup CB) on the device.  This module keeps the
winners in a JSON table so that a solve can use a measured schedule without tuning
again:

    python -m paper_0911_4498_amd.autotune 100000 50000 --write   # tune, store
    sched = autotune.lookup(100000, 50000)                          # {"fft_mp", ...} or None
    plan = ssa.Plan(N, L, k, **(sched or {}))

Each entry records the device it was measured on, the automatic schedule's time and the
best few candidates.  Any schedule gives the same products up to FP32 rounding (any
M >= N is exact, Sec. 4.2), so a table entry only changes speed.
"""
from __future__ import annotations

import argparse
import json
import os
import time

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fft_schedules.json")


def _key(N: int, L: int) -> str:
    return f"{int(N)}:{int(L)}"


def load_table(path: str = TABLE) -> dict:
    """The stored entries ({} if the file does not exist)."""
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        data = json.load(fh)
    if not isinstance(data, dict) or not isinstance(data.get("entries", {}), dict):
        raise ValueError(f"{path}: not a schedule table")
    return data.get("entries", {})


def lookup(N: int, L: int, path: str = TABLE) -> dict | None:
    """Plan keyword arguments {"fft_mp", "fft_m1", "fft_cb"} stored for (N, L), or None."""
    e = load_table(path).get(_key(N, L))
    if e is None:
        return None
    return {"fft_mp": int(e["fft_mp"]), "fft_m1": int(e["fft_m1"]), "fft_cb": int(e["fft_cb"])}


def tune(N: int, L: int, series=None, reps: int = 20, device=None) -> dict:
    """Run the tuner on the device and return a table entry (not stored)."""
    import torch

    from . import ssa
    t0 = time.perf_counter()
    best, us, table = ssa.tune_fft(N, L, series, reps=reps, device=device)
    dt = time.perf_counter() - t0
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    auto = table[0]
    top = sorted(table, key=lambda r: r[3])[:5]
    return {**best, "us_per_pair": round(us, 3),
            "auto": {"fft_mp": auto[0], "fft_m1": auto[1], "fft_cb": auto[2], "us_per_pair": round(auto[3], 3)},
            "top": [{"fft_mp": r[0], "fft_m1": r[1], "fft_cb": r[2], "us_per_pair": round(r[3], 3)} for r in top],
            "candidates": len(table), "reps": int(reps), "tune_s": round(dt, 3),
            "device": torch.cuda.get_device_name(dev)}


def store(N: int, L: int, entry: dict, path: str = TABLE) -> None:
    """Add or replace the entry of (N, L) in the table file."""
    entries = load_table(path)
    entries[_key(N, L)] = entry
    data = {"about": "FFT schedules of the single-series products chosen by ssa_tune_fft; "
                     "written by python -m paper_0911_4498_amd.autotune",
            "entries": dict(sorted(entries.items(), key=lambda kv: [int(x) for x in kv[0].split(":")]))}
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1)
        fh.write("\n")
    os.replace(tmp, path)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description="tune the FFT schedule of the products for (N, L) pairs")
    ap.add_argument("sizes", type=int, nargs="+", help="N L [N L ...]")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--write", action="store_true", help="store the results in the table")
    ap.add_argument("--table", default=TABLE)
    a = ap.parse_args(argv)
    if len(a.sizes) % 2:
        ap.error("sizes come in N L pairs")
    for N, L in zip(a.sizes[0::2], a.sizes[1::2]):
        e = tune(N, L, reps=a.reps)
        print(json.dumps({"N": N, "L": L, **e}), flush=True)
        if a.write:
            store(N, L, e, a.table)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
