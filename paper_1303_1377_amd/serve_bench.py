"""Serving trace on one GPU: Poisson arrivals of solve requests over six
resident gauge fields, against the plain FP64 one-at-a-time form.

    python -m paper_1303_1377_amd.serve_bench [--requests 200] [--loads 0.5,0.8,1.0]
        [--budget-gb 200] [--max-rhs 4] [--baseline-requests 12] [--small]

Fields (links exp(i 0.4 H) reunitarised to SU(3), two APE steps, csw 1; the
16^4 fields drawn on the host, the larger ones on the GPU):
  seeds 0, 1   16^4         two levels, aggregates / SAP blocks 4^4, N 20, m0 = m_crit + 0.02
  seeds 2, 3   48 x 24^3    three levels, aggregates 4^4 then 2^4, SAP blocks 4^4 then
                            2 x 3^3, coarsest 6 x 3^3 (plain GMRES), N 20 / 20, m0 = m_crit + 0.01
  seeds 4, 5   64 x 32^3    three levels, aggregates 4^4 then 2^4, N 20 / 20, m0 = m_crit + 0.01
with m_crit each field's own critical mass (paper_1303_1377_amd/mcrit_fields.json).
Preconditioner FP32 (mixed precision), FP64 outer FGMRES(10), tolerance 1e-10.

Requests: arrival times from a Poisson process (rate = load x the measured
capacity of the server), field uniform over the six, 1..12 Gaussian
right-hand sides (uniform), arrival seed 42; one trace per load.  The server
admits setups by the HBM budget (evicting idle ones), keeps every field's
setup resident, refills the slots of each field's outer FGMRES as right-hand
sides finish (continuous batching) and runs fields concurrently.  Reported
per load: p50 / p99 request latency (submit to result; the first trace
includes the cold setups), RHS solved per second.  The capacity is measured
in a closed loop on resident setups over the first requests; the baseline
solves the RHS of the same requests one at a time with an FP64 preconditioner
on resident setups, so the two solves/s figures compare the same work.
--small uses 8^4 / 16 x 8^3-size stand-ins for a quick functional run.
Prints one JSON line.
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
    with open(os.path.join(ROOT, "paper_1303_1377_amd", "mcrit_fields.json")) as f:
        mc = json.load(f)
    if small:
        base = mc["lat16x4_ape2_seed0"]["m_crit"]
        return [dict(seed=s, dims=d, m0=base + 0.02, levels=2, device=False) for s, d in
                ((0, (8, 8, 8, 8)), (1, (8, 8, 8, 8)), (2, (16, 8, 8, 8)), (3, (16, 8, 8, 8)), (4, (8, 8, 8, 16)),
                 (5, (8, 8, 8, 16)))]
    mcr = lambda key: mc[key]["m_crit"]
    return [dict(seed=0, dims=(16, 16, 16, 16), m0=mcr("lat16x4_ape2_seed0") + 0.02, levels=2, device=False),
            dict(seed=1, dims=(16, 16, 16, 16), m0=mcr("lat16x4_ape2_seed1") + 0.02, levels=2, device=False),
            dict(seed=2, dims=(48, 24, 24, 24), m0=mcr("lat48x24c3_ape2_seed2_dev") + 0.01, levels=3, device=True,
                 sap1=(2, 3, 3, 3)),
            dict(seed=3, dims=(48, 24, 24, 24), m0=mcr("lat48x24c3_ape2_seed3_dev") + 0.01, levels=3, device=True,
                 sap1=(2, 3, 3, 3)),
            dict(seed=4, dims=(64, 32, 32, 32), m0=mcr("lat64x32c3_ape2_seed4_dev") + 0.01, levels=3, device=True),
            dict(seed=5, dims=(64, 32, 32, 32), m0=mcr("lat64x32c3_ape2_seed5_dev") + 0.01, levels=3, device=True)]


def field_params(G, f, precision, max_rhs):
    # outer FGMRES(10): the FP64 Krylov basis of max_rhs RHS is the largest
    # part of a setup (with FGMRES(25) the six fields need about 250 GB at four
    # RHS slots, above the 200 GB budget)
    if f["levels"] == 3:
        return G.default_params(levels=3, n_tv=[20, 20], agg=[(4, 4, 4, 4), (2, 2, 2, 2)],
                                sap=[(4, 4, 4, 4), f.get("sap1", (2, 2, 2, 2))], mr_steps=[4, 4], precision=precision,
                                max_rhs=max_rhs, outer_restart=10)
    return G.default_params(levels=2, n_tv=[20], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], mr_steps=[3],
                            precision=precision, max_rhs=max_rhs, outer_restart=10)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--loads", default="0.5,0.8,1.0")
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
        if f["device"]:
            U[i] = F.make_gauge_device(f["dims"], 0.4, f["seed"], ape_steps=2, ape_alpha=0.5)
        else:
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
        """k complex Gaussian right-hand sides (re, im ~ N(0, 1)) drawn on the
        device from a seeded torch generator (a 64 x 32^3 one is 403 MB)."""
        d = table[fi]["dims"]
        g = torch.Generator(device="cuda")
        g.manual_seed(int(seed))
        re = torch.randn((k, d[0] * d[1] * d[2] * d[3], 4, 3), dtype=torch.float64, device="cuda", generator=g)
        im = torch.randn((k, d[0] * d[1] * d[2] * d[3], 4, 3), dtype=torch.float64, device="cuda", generator=g)
        return torch.complex(re, im)

    # capacity: time the batched server on a closed-loop burst of the first requests (setups excluded)
    srv = Server(budget_bytes=a.budget_gb * 1e9, max_rhs=a.max_rhs)
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
            if fu.exception() is not None:
                raise fu.exception()
        cap_s = time.time() - t0
        cap_rps = n_cap / cap_s
        cap_rhs = sum(k for _, k, _ in reqs[:n_cap])
        cap_sps = cap_rhs / cap_s
        futs = cap_data = None
    finally:
        srv.close()
    _log("serve_bench: capacity %.2f requests/s, %.2f RHS/s (closed loop, %d requests, %d RHS)" %
         (cap_rps, cap_sps, n_cap, cap_rhs))

    # one trace per load: Poisson arrivals at load x capacity; the first starts
    # cold.  Each request's right-hand sides are drawn on the device when it is
    # submitted; results are checked in the completion callback and dropped (the
    # device holds only the requests in flight)
    traces = []
    srv = Server(budget_bytes=a.budget_gb * 1e9, max_rhs=a.max_rhs)
    for i, f in enumerate(table):
        srv.add_field(i, f["dims"], U[i], f["m0"], 1.0, params=field_params(G, f, a.precision, a.max_rhs))
    worst = [0.0]
    try:
        for li, load in enumerate(float(v) for v in a.loads.split(",")):
            rate = load * cap_rps
            gaps = np.random.default_rng(43 + li).exponential(1.0 / rate, size=len(reqs))
            lock = threading.Lock()
            lat = []
            errors = []
            all_done = threading.Event()

            def done(fu, t_sub, lat=lat, errors=errors, all_done=all_done):
                exc = fu.exception()
                with lock:
                    if exc is not None:
                        errors.append(exc)
                    else:
                        worst[0] = max(worst[0], max(s_["true_relres"] for s_ in fu.result()[1]))
                    lat.append(time.time() - t_sub)
                    n = len(lat)
                    if n % 10 == 0:
                        _log("serve_bench: load %.1f: %d of %d requests done" % (load, n, len(reqs)))
                    if n == len(reqs):
                        all_done.set()

            t_start = time.time()
            n_rhs = 0
            for (fi, k, s), gap in zip(reqs, gaps):
                time.sleep(gap)
                b = rhs(fi, k, s)
                torch.cuda.synchronize()
                t_sub = time.time()
                fu = srv.submit(fi, b)
                fu.add_done_callback(lambda f_, t_sub=t_sub: done(f_, t_sub))
                del fu, b
                n_rhs += k
            all_done.wait()
            wall = time.time() - t_start
            if errors:
                raise errors[0]
            st = srv.stats()
            lat_a = np.array(lat)
            traces.append(dict(load=load, arrival_rate_per_s=rate, wall_s=wall, requests=len(reqs), rhs=n_rhs,
                               p50_latency_s=float(np.percentile(lat_a, 50)),
                               p99_latency_s=float(np.percentile(lat_a, 99)),
                               rhs_per_s=n_rhs / wall, cold_start=(li == 0), admitted=st["admitted"],
                               evicted=st["evicted"], resident_gb=st["resident_bytes"] / 1e9))
            _log("serve_bench: trace at load %.1f: %s" % (load, traces[-1]))
    finally:
        srv.close()
    worst = worst[0]

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
        B = rhs(fi, k, s)
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
               requests_per_trace=len(reqs), max_rhs=a.max_rhs, budget_gb=a.budget_gb, precision=a.precision,
               true_relres_max=worst, capacity_requests_per_s=cap_rps, capacity_solves_per_s=cap_sps,
               capacity_rhs=cap_rhs, traces=traces,
               baseline_fp64_one_at_a_time_solves_per_s=base_sps, baseline_rhs=n_rhs,
               capacity_vs_baseline=cap_sps / base_sps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
