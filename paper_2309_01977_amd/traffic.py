"""HBM traffic per kernel launch from two rocprofv3 counter runs.

    python -m paper_2309_01977_amd.traffic FETCH.csv WRITE.csv > traffic.json

The inputs are the counter_collection.csv files of
    rocprofv3 --pmc FETCH_SIZE ... -- python3 bench.py --recon-only --steps 1 --warmup 0
    rocprofv3 --pmc WRITE_SIZE ... -- python3 bench.py --recon-only --steps 1 --warmup 0
FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what the same
counters read for one plain device copy of known size (the 256 MiB copy
that bench.py performs before the data are generated), and averaged over the
launches that belong to the reconstruction: every dispatch after the first
fwd_reduce (the data generation before it is one forward pass over all
angles, which ends with that reduction).  The result is keyed to a digest of the kernel sources; bench.py
reports it only while the sources are unchanged.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
COPY_KIB = 256 * 1024


def source_digest() -> str:
    """sha256 over every kernel source file, in name order."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()


def _base(kernel_name: str) -> str:
    n = re.sub(r"\(anonymous namespace\)::", "", kernel_name).replace("void ", "")
    n = n.split("(")[0].split("<")[0]
    return n.split("::")[-1]


def _rows(path: str, counter: str):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows


def per_launch(path: str, counter: str):
    """(copy KiB, {kernel: [KiB per reconstruction dispatch]})."""
    rows = _rows(path, counter)
    copy = [float(r["Counter_Value"]) for r in rows
            if "copyBuffer" in r["Kernel_Name"] and int(r["Grid_Size"]) >= 65536]
    if not copy:
        raise SystemExit(f"{path}: no calibration copy found")
    start = 1 + next(i for i, r in enumerate(rows) if _base(r["Kernel_Name"]) == "fwd_reduce")
    out = defaultdict(list)
    for r in rows[start:]:
        if "spectk" in r["Kernel_Name"]:
            out[_base(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return copy[0], out


def summarise(fetch_csv: str, write_csv: str) -> dict:
    fc, f = per_launch(fetch_csv, "FETCH_SIZE")
    wc, w = per_launch(write_csv, "WRITE_SIZE")
    kf, kw = COPY_KIB / fc, COPY_KIB / wc
    out = {"source_sha256": source_digest(), "fetch_scale": kf, "write_scale": kw,
           "copy_fetch_KiB": fc, "copy_write_KiB": wc, "kernels": {}}
    for k in sorted(set(f) | set(w)):
        fv, wv = f.get(k, [0.0]), w.get(k, [0.0])
        fk, wk = sum(fv) / len(fv), sum(wv) / len(wv)
        out["kernels"][k] = {"launches": len(fv), "fetch_KiB_raw": fk, "write_KiB_raw": wk,
                             "hbm_bytes_per_launch": (fk * kf + wk * kw) * 1024}
    return out


if __name__ == "__main__":
    print(json.dumps(summarise(sys.argv[1], sys.argv[2]), indent=1))
