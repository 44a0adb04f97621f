"""Serving trace on one GPU: Poisson arrivals of solve requests over six
resident gauge fields, against the plain FP64 one-at-a-time form.

    python -m paper_1303_1377_amd.serve_bench [--requests 60] [--load 0.8]
        [--budget-gb 200] [--max-rhs 4] [--baseline-requests 12] [--small]

Fields (links exp(i 0.4 H) reunitarised to SU(3), two APE steps, csw 1):
  seeds 0, 1   16^4           two levels, aggregates / SAP blocks 4^4, N 20
  seeds 2, 3   48 x 24^3      two levels, aggregates / SAP blocks 4^4, N 20
  seeds 4, 5   64 x 32^3      three levels, aggregates 4^4 then 2^4, N 20 / 20
m0 = m_crit + 0.02 (16^4) or + 0.01 (larger lattices), m_crit from
tests/golden/mcrit.json (the 16^4 seed-0 value where no other is stored).
Preconditioner FP32 (mixed precision) or FP16 storage, FP64 outer FGMRES(10),
tolerance 1e-10.

Requests: arrival times from a Poisson process (rate = load x the measured
capacity of the batched server), field uniform over the six, 1..12 Gaussian
right-hand sides (uniform), arrival seed 42.  The server admits setups by the
HBM budget (evicting idle ones), batches RHS per field up to max_rhs and runs
fields concurrently.  Reported: p50 / p99 request latency (submit to result,
cold setups included), RHS solved per second; the baseline solves the RHS of
the same first requests one at a time with an FP64 preconditioner on resident
setups; the served form's capacity is measured on those requests in a closed
loop on resident setups, so the two solves/s figures compare the same work.  --small uses 8^4 / 8x4^3-size
stand-ins for a quick functional run.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def field_table(small=False):
    with open(os.path.join(ROOT, "tests", "golden", "mcrit.json")) as f:
        mc = json.load(f)
    base = mc["lat16x4_ape2_seed0"]["m_crit"]
    c3 = mc.get("lat64x32c3_ape2_seed0", {}).get("m_crit", base)
    if small:
        return [dict(seed=s, dims=d, m0=base + 0.02, levels=2) for s, d in
                ((0, (8, 8, 8, 8)), (1, (8, 8, 8, 8)), (2, (16, 8, 8, 8)), (3, (16, 8, 8, 8)), (4, (8, 8, 8, 16)),
                 (5, (8, 8, 8, 16)))]
    return [dict(seed=0, dims=(16, 16, 16, 16), m0=base + 0.02, levels=2),
            dict(seed=1, dims=(16, 16, 16, 16), m0=base + 0.02, levels=2),
            dict(seed=2, dims=(48, 24, 24, 24), m0=base + 0.01, levels=2),
            dict(seed=3, dims=(48, 24, 24, 24), m0=base + 0.01, levels=2),
            dict(seed=4, dims=(64, 32, 32, 32), m0=c3 + 0.01, levels=3),
            dict(seed=5, dims=(64, 32, 32, 32), m0=c3 + 0.01, levels=3)]


def field_params(G, f, precision, max_rhs):
    # outer FGMRES(10): the FP64 Krylov basis of max_rhs RHS is the largest
    # part of a setup (with FGMRES(25) the six fields need about 250 GB at four
    # RHS slots, above the 200 GB budget, and the server would evict setups in
    # the middle of the capacity run)
    if f["levels"] == 3:
        return G.default_params(levels=3, n_tv=[20, 20], agg=[(4, 4, 4, 4), (2, 2, 2, 2)],
                                sap=[(4, 4, 4, 4), (2, 2, 2, 2)], mr_steps=[4, 4], precision=precision, max_rhs=max_rhs,
                                outer_restart=10)
    return G.default_params(levels=2, n_tv=[20], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], mr_steps=[3],
                            precision=precision, max_rhs=max_rhs, outer_restart=10)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=60)
    ap.add_argument("--load", type=float, default=0.8)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--max-rhs", type=int, default=4)
    ap.add_argument("--baseline-requests", type=int, default=12,
                    help="requests (from the start of the trace) of the closed-loop capacity and baseline runs")
    ap.add_argument("--precision", type=int, default=32, help="preconditioner precision of the served setups")
    ap.add_argument("--small", action="store_true")
    a = ap.parse_args()

    import numpy as np
    import torch

    import paper_1303_1377_amd as G
    from paper_1303_1377_amd import fields as F
    from paper_1303_1377_amd.serving import Server

    table = field_table(a.small)
    t0 = time.time()
    U = {}
    for i, f in enumerate(table):
        U[i] = F.make_gauge(f["dims"], 0.4, f["seed"], ape_steps=2, ape_alpha=0.5)
        _log("serve_bench: field %d (%s, seed %d) generated at %.1fs" % (i, "x".join(map(str, f["dims"])), f["seed"],
                                                                         time.time() - t0))

    rng = np.random.default_rng(42)
    reqs = []
    for r in range(a.requests):
        fi = int(rng.integers(0, len(table)))
        k = int(rng.integers(1, 13))
        reqs.append((fi, k, 10000 + 37 * r))

    def rhs(fi, k, seed):
        return F.gaussian_spinor(table[fi]["dims"], seed, nrhs=k)

    # capacity: time the batched server on a closed-loop burst of the first requests (setups excluded)
    srv = Server(budget_bytes=a.budget_gb * 1e9, max_rhs=a.max_rhs, results_on_host=True)
    for i, f in enumerate(table):
        srv.add_field(i, f["dims"], U[i], f["m0"], 1.0, params=field_params(G, f, a.precision, a.max_rhs))
    try:
        warm = [srv.submit(i, rhs(i, 1, 5 + i)) for i in range(len(table))]
        for w in warm:
            w.result()
        _log("serve_bench: all six setups resident or evicted after warm-up")
        n_cap = min(len(reqs), a.baseline_requests)
        cap_data = [rhs(fi, k, s) for fi, k, s in reqs[:n_cap]]
        t0 = time.time()
        futs = [srv.submit(fi, b) for (fi, k, s), b in zip(reqs[:n_cap], cap_data)]
        for fu in futs:
            fu.exception()
        cap_s = time.time() - t0
        cap_rps = n_cap / cap_s
        cap_rhs = sum(k for _, k, _ in reqs[:n_cap])
        cap_sps = cap_rhs / cap_s
        futs = cap_data = None
    finally:
        srv.close()
    _log("serve_bench: capacity %.2f requests/s, %.2f RHS/s (closed loop, %d requests, %d RHS)" %
         (cap_rps, cap_sps, n_cap, cap_rhs))

    # the trace: Poisson arrivals at load x capacity, cold start
    rate = a.load * cap_rps
    gaps = np.random.default_rng(43).exponential(1.0 / rate, size=len(reqs))
    srv = Server(budget_bytes=a.budget_gb * 1e9, max_rhs=a.max_rhs, results_on_host=True)
    for i, f in enumerate(table):
        srv.add_field(i, f["dims"], U[i], f["m0"], 1.0, params=field_params(G, f, a.precision, a.max_rhs))
    # right-hand sides are drawn on the host before the trace; the server copies
    # each batch to the device when it runs and returns results to the host
    # (a 64 x 32^3 RHS is 403 MB: the device holds only the batches in flight)
    host = []
    for n, (fi, k, s) in enumerate(reqs):
        host.append(F.gaussian_spinor(table[fi]["dims"], s, nrhs=k))
        if n % 10 == 9:
            _log("serve_bench: %d right-hand-side sets drawn" % (n + 1))
    worst = [0.0]
    ndone = [0]
    lock = threading.Lock()

    def done(fu):
        x, st = fu.result()
        with lock:
            worst[0] = max(worst[0], max(s_["true_relres"] for s_ in st))
            ndone[0] += 1
            _log("serve_bench: request %d of %d done (%d RHS)" % (ndone[0], len(reqs), len(st)))

    try:
        t_start = time.time()
        futs = []
        for (fi, k, s), b, gap in zip(reqs, host, gaps):
            time.sleep(gap)
            fu = srv.submit(fi, b)
            fu.add_done_callback(done)
            futs.append(fu)
        for fu in futs:
            fu.exception()
        wall = time.time() - t_start
        stats = srv.stats()
    finally:
        srv.close()
    futs = None
    worst = worst[0]
    _log("serve_bench: trace done in %.1fs %s" % (wall, stats))

    # baseline: FP64 preconditioner, one RHS at a time, resident setups (setup excluded)
    nb = min(a.baseline_requests, len(reqs))
    solvers = {}
    n_rhs = 0
    t_solve = 0.0
    for fi, k, s in reqs[:nb]:
        if fi not in solvers:
            f = table[fi]
            sv = G.Solver(f["dims"], U[fi], f["m0"], 1.0)
            sv.setup(params=field_params(G, f, 64, 1))
            if len(solvers) >= 2:   # keep at most three FP64 setups resident
                old = next(iter(solvers))
                solvers.pop(old).close()
            solvers[fi] = sv
        B = torch.as_tensor(rhs(fi, k, s)).to("cuda")
        torch.cuda.synchronize()
        t0 = time.time()
        for q in range(k):
            solvers[fi].solve(B[q], 1e-10)
        torch.cuda.synchronize()
        t_solve += time.time() - t0
        n_rhs += k
        _log("serve_bench: baseline %d RHS solved" % n_rhs)
    for sv in solvers.values():
        sv.close()
    base_sps = n_rhs / t_solve
    _log("serve_bench: FP64 one-at-a-time %.2f solves/s over %d RHS" % (base_sps, n_rhs))
    out = dict(metric="serving p50/p99 latency and solves/s", fields=[dict(seed=f["seed"], dims=list(f["dims"]),
                                                                          m0=f["m0"], levels=f["levels"]) for f in table],
               requests=len(reqs), load=a.load, arrival_rate_per_s=rate, capacity_requests_per_s=cap_rps,
               max_rhs=a.max_rhs, budget_gb=a.budget_gb, wall_s=wall, true_relres_max=worst,
               p50_latency_s=stats["p50_latency_s"], p99_latency_s=stats["p99_latency_s"],
               solves_per_s=stats["solves_per_s"], requests_per_s=stats["requests_per_s"],
               admitted=stats["admitted"], evicted=stats["evicted"],
               capacity_solves_per_s=cap_sps, capacity_rhs=cap_rhs,
               baseline_fp64_one_at_a_time_solves_per_s=base_sps, baseline_rhs=n_rhs,
               capacity_vs_baseline=cap_sps / base_sps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
