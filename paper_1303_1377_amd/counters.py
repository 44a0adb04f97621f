"""Reduce rocprofv3 counter-collection CSVs to per-kernel means and write the
counter record bench.py reads for its roofline `traffic` figure.

    python -m paper_1303_1377_amd.counters --fetch DIR_FETCH --write DIR_WRITE \\
        --out profiles/counters_16x4_fp64_solve.json --command "..."

Each DIR holds the *_counter_collection.csv of one `rocprofv3 --pmc` run
(FETCH_SIZE, then WRITE_SIZE, in KiB per dispatch).  Kernels are matched by
name to the library's kernel classes; the record stores, per class, the mean
counter values, the number of dispatches, and the SHA-256 of the source file
that holds the kernel (a later change of that file voids the record).  The
scale factors turn the counters into bytes: FETCH_SIZE reads half of what a
plain copy kernel provably reads on MI355X (x2.0), WRITE_SIZE reads exactly
its writes (x1.0).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# kernel class -> (kernel name prefix in the trace, source file)
CLASSES = {
    "sap": ("void dd::k_sap_fine<double, double, 1>(", "paper_1303_1377_amd/csrc/dd_fine.hip"),
    "dirac64": ("void dd::k_dirac<double, double>(", "paper_1303_1377_amd/csrc/dd_fine.hip"),
    "restrict": ("void dd::k_restrict_fine<double, double, 256>(", "paper_1303_1377_amd/csrc/dd_fine.hip"),
    "prolong": ("void dd::k_prolong_fine<double, double>(", "paper_1303_1377_amd/csrc/dd_fine.hip"),
}


def per_kernel(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    vals = {}
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return vals


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--command", default="")
    a = ap.parse_args()
    fe, wr = per_kernel(a.fetch), per_kernel(a.write)
    rec = dict(fetch_scale=2.0, write_scale=1.0, command=a.command, kernels={})
    for cls, (prefix, src) in CLASSES.items():
        fk = [v for n, vs in fe.items() if n.startswith(prefix) for v in vs]
        wk = [v for n, vs in wr.items() if n.startswith(prefix) for v in vs]
        if not fk or not wk:
            continue
        with open(os.path.join(ROOT, src), "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
        rec["kernels"][cls] = dict(kernel=prefix, fetch_kib=sum(fk) / len(fk), write_kib=sum(wk) / len(wk),
                                   dispatches=min(len(fk), len(wk)), source=src, source_sha256=digest)
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
