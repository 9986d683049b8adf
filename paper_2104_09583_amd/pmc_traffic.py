"""HBM traffic per dispatch from two rocprofv3 counter runs of bench.py.

Takes the counter-collection CSVs of a FETCH_SIZE run and of a WRITE_SIZE run
(same bench command, kernels filtered to the measured kernel and the
reference copy), scales each counter by what it reads for the reference copy
of known size (bench.py ends with one copy of 256 MiB, read and written once),
and writes, per kernel, the mean HBM bytes per dispatch over the dispatches of
the timed steps (the last launches_per_step * steps dispatches, from the
bench JSON line of the same run; for the default workload bench.py runs with
--no-plain, so that no other launches follow them) beside the algorithmic bytes per dispatch
that bench.py measured, keyed by the sha256 of the kernel source so that a
stale summary is not used.

    python -m paper_2104_09583_amd.pmc_traffic --fetch F.csv --write W.csv \
        --bench bench.json --kind bconv_colpass --regex ntt_bridge_kernel --out profiles/X.json
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re

CALIB_BYTES = 256 << 20
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def read_counter(path: str, counter: str):
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--bench", required=True, help="the bench.py JSON line of the counter run")
    ap.add_argument("--kind", required=True, help="kernel class name as in bench.py's kernels section")
    ap.add_argument("--regex", required=True, help="kernel-name pattern of that class")
    ap.add_argument("--command", action="append", default=[], help="the commands that made the CSVs")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    with open(a.bench) as f:
        bench = json.loads(f.read().strip().splitlines()[-1])
    k = bench["kernels"][a.kind]
    n = int(round(k["launches_per_step"] * bench["steps"]))
    out = {"workload": bench["config"]["workload"], "kind": a.kind, "kernel_regex": a.regex,
           "commands": a.command}
    with open(os.path.join(ROOT, "paper_2104_09583_amd", "csrc", "kernels.hip"), "rb") as f:
        out["kernels_hip_sha256"] = hashlib.sha256(f.read()).hexdigest()
    per = {}
    for name, path, counter in (("fetch", a.fetch, "FETCH_SIZE"), ("write", a.write, "WRITE_SIZE")):
        rows = read_counter(path, counter)
        calib = [v for _, kn, v in rows if "calib_copy" in kn]
        if not calib:
            raise SystemExit(f"{path}: no reference copy dispatch")
        scale = CALIB_BYTES / (calib[-1] * 1024.0)
        sel = [v for _, kn, v in rows if re.search(a.regex, kn) and "calib_copy" not in kn]
        if len(sel) < n:
            raise SystemExit(f"{path}: {len(sel)} dispatches of {a.regex}, expected at least {n}")
        timed = sel[-n:]
        out[f"{name}_scale"] = scale
        per[name] = scale * 1024.0 * sum(timed) / n
    out["dispatches"] = n
    out["fetch_bytes_per_dispatch"] = round(per["fetch"])
    out["write_bytes_per_dispatch"] = round(per["write"])
    out["bytes_per_dispatch"] = round(per["fetch"] + per["write"])
    out["algorithmic_bytes_per_dispatch"] = round(k["algorithmic_bytes_per_launch"])
    out["measured_over_algorithmic"] = round(out["bytes_per_dispatch"] / max(1, k["algorithmic_bytes_per_launch"]), 4)
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
