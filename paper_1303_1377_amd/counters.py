"""Reduce rocprofv3 output: counter-collection CSVs to the counter record
bench.py reads for its roofline `traffic` figure, and kernel traces to
per-kernel statistics.

    python -m paper_1303_1377_amd.counters --fetch DIR_FETCH --write DIR_WRITE \\
        --out profiles/counters_48c96_fp32_batch4.json --last 52 --command "..."
    python -m paper_1303_1377_amd.counters --stats RESULTS.db [--last-seconds T] [--top 20]

--last N keeps the last N dispatches of each class (the timed part of a run
that ends with it).  --stats reads the SQLite results database of `rocprofv3 --kernel-trace` and
prints calls, total, mean and share per kernel; --last-seconds keeps only the
dispatches that start in the last T seconds of GPU activity (the timed region
of a benchmark that ends with it).

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

# kernel class -> (kernel name prefixes in the trace, source file); the
# prefixes cover the FP64 and the FP32 forms of each class
CLASSES = {
    "sap": (("void dd::k_sap_fine<double, double, dd::cx<double>*, 1>(",
             "void dd::k_sap_fine<float, float, dd::cx<float>*, 2>(",
             "void dd::k_sap_fine<double, double, 1>("), "paper_1303_1377_amd/csrc/dd_fine.hip"),
    "dirac64": (("void dd::k_dirac<double, double", "void dd::k_dirac_lds<double, double"),
                "paper_1303_1377_amd/csrc/dd_fine.hip"),
    "restrict": (("void dd::k_restrict_fine<double, double, 256",
                  "void dd::k_restrict_fine<float, float, 256"), "paper_1303_1377_amd/csrc/dd_fine.hip"),
    "prolong": (("void dd::k_prolong_fine<double, double", "void dd::k_prolong_fine<float, float"),
                "paper_1303_1377_amd/csrc/dd_fine.hip"),
}


def per_kernel(d):
    """Counter values per kernel name, in dispatch order."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    rows = []
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
    vals = {}
    for _, name, v in sorted(rows):
        vals.setdefault(name, []).append(v)
    return vals


def kernel_stats(db, last_seconds=None, top=20):
    """Per-kernel (calls, total us, mean us, share) from a rocprofv3 SQLite results file."""
    import sqlite3

    c = sqlite3.connect(db)
    rows = list(c.execute("select name, start, end from kernels"))
    if last_seconds:
        t_end = max(r[2] for r in rows)
        rows = [r for r in rows if r[1] >= t_end - last_seconds * 1e9]
    agg = {}
    for name, t0, t1 in rows:
        a = agg.setdefault(name, [0, 0.0])
        a[0] += 1
        a[1] += (t1 - t0) / 1e3
    tot = sum(v[1] for v in agg.values())
    out = sorted(((n, v[0], v[1], v[1] / v[0], 100.0 * v[1] / tot) for n, v in agg.items()), key=lambda r: -r[2])
    return out[:top], tot, len(rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--out")
    ap.add_argument("--command", default="")
    ap.add_argument("--stats")
    ap.add_argument("--last-seconds", type=float, default=None)
    ap.add_argument("--top", type=int, default=20)
    ap.add_argument("--last", type=int, default=None,
                    help="keep the last N dispatches of each class (the timed part of a run that ends with it)")
    a = ap.parse_args()
    if a.stats:
        rows, tot, n = kernel_stats(a.stats, a.last_seconds, a.top)
        print("%d dispatches, %.1f us of kernel time" % (n, tot))
        print("| kernel | calls | total (us) | average (us) | % |")
        print("|---|---|---|---|---|")
        for name, calls, t, avg, pct in rows:
            print("| `%s` | %d | %.1f | %.2f | %.2f |" % (name[:100] + ("..." if len(name) > 100 else ""), calls, t, avg, pct))
        return
    fe, wr = per_kernel(a.fetch), per_kernel(a.write)
    rec = dict(fetch_scale=2.0, write_scale=1.0, command=a.command, kernels={})
    for cls, (prefixes, src) in CLASSES.items():
        prefix = next((p for p in prefixes if any(n.startswith(p) for n in fe)), None)
        if prefix is None:
            continue
        fk = [v for n, vs in fe.items() if n.startswith(prefix) for v in vs]
        wk = [v for n, vs in wr.items() if n.startswith(prefix) for v in vs]
        if a.last:
            fk, wk = fk[-a.last:], wk[-a.last:]
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
