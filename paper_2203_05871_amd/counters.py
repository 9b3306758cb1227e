"""Digest of rocprofv3 counter passes into per-launch figures of one kernel.

rocprofv3 writes one CSV row per (dispatch, counter) with `--pmc C -f csv`.
This module sums each counter per dispatch, takes a window of the kernel's
dispatches (the last `window` of them before `skip_tail` more, in dispatch
order: the timed steps of a benchmark run), averages it, and scales
FETCH_SIZE / WRITE_SIZE by what the same counter reads for a plain device
copy of known size in the same run (the largest `copyBuffer` dispatch).

    python -m paper_2203_05871_amd.counters --kernel svd_persistent_kernel \
        --pass FETCH_SIZE=fetch.csv --pass WRITE_SIZE=write.csv --copy-kib 262144 \
        --window 3500 --skip-tail 3500 --workload "..." --source a.hip ... --out x.json
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys
from collections import defaultdict


def per_dispatch(path):
    """{dispatch id: (kernel name, {counter: summed value})} of one CSV."""
    out = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            d = int(row["Dispatch_Id"])
            name = row["Kernel_Name"]
            ent = out.setdefault(d, (name, defaultdict(float)))
            ent[1][row["Counter_Name"]] += float(row["Counter_Value"])
    return out


def window_mean(disp, kernel, counter, window, skip_tail):
    ids = sorted(d for d, (n, c) in disp.items() if kernel in n and counter in c)
    if skip_tail:
        ids = ids[:len(ids) - skip_tail]
    if window:
        ids = ids[-window:]
    if not ids:
        raise SystemExit(f"no dispatches of {kernel} with {counter}")
    vals = [disp[d][1][counter] for d in ids]
    return sum(vals) / len(vals), len(vals), len([d for d, (n, c) in disp.items() if kernel in n])


def copy_reading(disp, counter):
    vals = [c[counter] for d, (n, c) in disp.items() if "copyBuffer" in n and counter in c]
    return max(vals) if vals else None


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--kernel", required=True, help="substring of the kernel name")
    ap.add_argument("--pass", dest="passes", action="append", default=[], metavar="COUNTER=CSV")
    ap.add_argument("--window", type=int, default=0, help="dispatches averaged (0: all)")
    ap.add_argument("--skip-tail", type=int, default=0, help="dispatches after the window")
    ap.add_argument("--copy-kib", type=float, default=0.0, help="size of the calibration copy, KiB")
    ap.add_argument("--workload", default="")
    ap.add_argument("--command", action="append", default=[], help="the profiling commands, for the record")
    ap.add_argument("--source", action="append", default=[], help="kernel sources to hash (repo-relative)")
    ap.add_argument("--root", default=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)
    rec = {"kernel": a.kernel, "workload": a.workload, "commands": a.command}
    hbm = 0.0
    have_fetch = have_write = False
    for item in a.passes:
        counter, path = item.split("=", 1)
        disp = per_dispatch(path)
        mean, n, total = window_mean(disp, a.kernel, counter, a.window, a.skip_tail)
        rec[f"{counter}_per_launch_raw"] = mean
        rec["launches_averaged"] = n
        rec["launches_in_run"] = total
        if counter in ("FETCH_SIZE", "WRITE_SIZE") and a.copy_kib > 0:
            cp = copy_reading(disp, counter)
            if cp:
                scale = a.copy_kib / cp
                rec[f"{counter}_copy_reading_kib"] = cp
                rec[f"{counter}_scale"] = scale
                hbm += mean * scale * 1024.0
                have_fetch |= counter == "FETCH_SIZE"
                have_write |= counter == "WRITE_SIZE"
    if have_fetch and have_write:
        rec["hbm_bytes_per_launch"] = hbm
    if a.source:
        h = hashlib.sha256()
        for rel in a.source:
            with open(os.path.join(a.root, rel), "rb") as f:
                h.update(f.read())
        rec["sources"] = a.source
        rec["source_sha256"] = h.hexdigest()
    text = json.dumps(rec, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    print(text)


if __name__ == "__main__":
    sys.exit(main())
