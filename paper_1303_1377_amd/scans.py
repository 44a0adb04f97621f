"""Synthetic replicas of the paper's parameter scans on the 16^4 workload.

    python -m paper_1303_1377_amd.scans [--dims 16,16,16,16] [--solves 2]

Field: links exp(i 0.4 H) reunitarised to SU(3), two APE steps (alpha 0.5),
seed 0, csw 1 (the benchmarked field; m_crit from tests/golden/mcrit.json).
Two-level FP64 DD-alphaAMG with the benchmark's parameters (aggregates and SAP
blocks 4^4, N = 20, 3 MR steps, nu = 2, coarsest odd-even GMRES(30) to 5e-2,
outer FGMRES(25) to 1e-10), Gaussian right-hand sides.

  n_inv scan (the setup/solve trade-off, Sec. 6 / Table 4): setup time and
      time to solution for n_inv = 1, 2, 3, 4, 6 at m_crit + 0.02.
  mass scan (one setup for several masses, Sec. 6 / Table 6): one setup at
      m_crit + 0.02 reused through dd_set_mass for m0 = m_crit + shift, against
      a fresh setup at every mass; outer and coarse iterations and times.

  inexact-deflation comparison (Sec. 6, Tables 8 and 9), `--scan id`: for
      n_inv = 1, 2, 3, 4, 5, 6, 8, 10 the setup time, outer iterations, mean
      coarse iterations per outer iteration and time to solution of inexact
      deflation (its own setup of Sec. 4.3, nu = 5, coarse systems to 1e-12)
      beside DD-alphaAMG (Algorithm 2, nu = 2, coarse 5e-2), both two-level
      FP64 on the same field, the same aggregates and N = 20.  Lattices other
      than 16^4 take their field on the device (--device-field) and their
      m_crit from mcrit_fields.json.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SHIFTS = (0.1, 0.05, 0.02, 0.01, 0.005, 0.002)
NINV = (1, 2, 3, 4, 6)


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def params(G, n_inv=6):
    return G.default_params(levels=2, n_tv=[20], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], mr_steps=[3], nu=2,
                            n_inv=n_inv, coarse_tol=5e-2, coarse_restart=30, outer_restart=25, precision=64)


def solve_stats(torch, s, B, tol=1e-10):
    times, outer, coarse, res = [], [], [], []
    for b in B:
        torch.cuda.synchronize()
        t = time.time()
        x, st = s.solve(b, tol)
        torch.cuda.synchronize()
        times.append(time.time() - t)
        outer.append(st["outer_iters"])
        coarse.append(st["coarse_iters"][1])
        res.append(st["true_relres"])
    return dict(time_to_solution_s=min(times), outer_iters=outer, coarse_iters=coarse, true_relres_max=max(res))


ID_NINV = (1, 2, 3, 4, 5, 6, 8, 10)


def id_scan(a, dims):
    import torch

    import paper_1303_1377_amd as G
    from paper_1303_1377_amd import fields as F

    with open(os.path.join(ROOT, "paper_1303_1377_amd", "mcrit_fields.json")) as f:
        mc = json.load(f)
    key = "lat%s_ape2_seed0%s" % ("16x4" if dims == (16, 16, 16, 16) else "%dx%dc3" % (dims[0], dims[1]),
                                  "_dev" if a.device_field else "")
    m_crit = mc[key]["m_crit"]
    m0 = m_crit + a.shift
    if a.device_field:
        U = F.make_gauge_device(dims, 0.4, 0, ape_steps=2, ape_alpha=0.5)
    else:
        U = F.make_gauge(dims, 0.4, 0, ape_steps=2, ape_alpha=0.5)
    B = [torch.as_tensor(F.gaussian_spinor(dims, 3000 + i)).to("cuda") for i in range(a.solves)]
    out = dict(dims=list(dims), field=key, m_crit=m_crit, m0=m0, solves=a.solves, tol=1e-10, id_coarse_tol=1e-12,
               points=[])

    def run(n_inv, method):
        s = G.Solver(dims, U, m0, 1.0)
        kw = dict(nu=5, id_setup=1) if method == "id" else dict(nu=2)
        p = G.default_params(levels=2, n_tv=[20], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], mr_steps=[3], n_inv=n_inv,
                             coarse_tol=5e-2, coarse_restart=30, coarse_maxit=5000, outer_restart=25, precision=64,
                             **kw)
        torch.cuda.synchronize()
        t = time.time()
        s.setup(params=p)
        torch.cuda.synchronize()
        setup_s = time.time() - t
        s.autotune(reps=2)
        if method == "dd":
            s.autotune_coarse(reps=1)
        times, outer, coarse, res = [], [], [], []
        for b in B:
            torch.cuda.synchronize()
            t = time.time()
            if method == "id":
                _, st = s.solve_id(b, 1e-10, nu=5, coarse_tol=1e-12)
            else:
                _, st = s.solve(b, 1e-10)
            torch.cuda.synchronize()
            times.append(time.time() - t)
            outer.append(st["outer_iters"])
            coarse.append(st["coarse_iters"][1] / max(st["outer_iters"], 1))
            res.append(st["true_relres"])
        s.close()
        r = dict(setup_s=setup_s, time_to_solution_s=min(times), outer_iters=outer,
                 coarse_iters_per_outer=[round(c, 1) for c in coarse], true_relres_max=max(res))
        _log("scans: %s n_inv %d setup %.3fs TTS %.4fs outer %s coarse/outer %s relres %.1e" %
             (method, n_inv, setup_s, r["time_to_solution_s"], outer, r["coarse_iters_per_outer"], max(res)))
        return r

    for n in ID_NINV:
        out["points"].append(dict(n_inv=n, id=run(n, "id"), dd=run(n, "dd")))
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", default="16,16,16,16")
    ap.add_argument("--solves", type=int, default=2)
    ap.add_argument("--scan", choices=("ninv_mass", "id"), default="ninv_mass")
    ap.add_argument("--device-field", action="store_true")
    ap.add_argument("--shift", type=float, default=0.02, help="m0 - m_crit (--scan id)")
    a = ap.parse_args()
    dims = tuple(int(v) for v in a.dims.split(","))
    if a.scan == "id":
        return id_scan(a, dims)

    import torch

    import paper_1303_1377_amd as G
    from paper_1303_1377_amd import fields as F

    with open(os.path.join(ROOT, "tests", "golden", "mcrit.json")) as f:
        m_crit = json.load(f)["lat16x4_ape2_seed0"]["m_crit"]
    U = F.make_gauge(dims, 0.4, 0, ape_steps=2, ape_alpha=0.5)
    B = [torch.as_tensor(F.gaussian_spinor(dims, 3000 + i)).to("cuda") for i in range(a.solves)]
    out = dict(dims=list(dims), m_crit=m_crit, solves=a.solves)

    def setup(m0, n_inv=6):
        s = G.Solver(dims, U, m0, 1.0)
        torch.cuda.synchronize()
        t = time.time()
        s.setup(params=params(G, n_inv))
        torch.cuda.synchronize()
        st = time.time() - t
        s.autotune(reps=2)
        s.autotune_coarse(reps=1)
        return s, st

    # n_inv scan
    ninv = []
    for n in NINV:
        s, st = setup(m_crit + 0.02, n)
        r = solve_stats(torch, s, B)
        r.update(n_inv=n, setup_s=st)
        ninv.append(r)
        _log("scans: n_inv %d setup %.3fs TTS %.4fs outer %s" % (n, st, r["time_to_solution_s"], r["outer_iters"]))
        s.close()
    out["n_inv_scan"] = ninv

    # mass scan: one setup reused, against a fresh setup per mass
    base, base_setup = setup(m_crit + 0.02)
    mass = []
    for sh in SHIFTS:
        m0 = m_crit + sh
        base.set_mass(m0)
        reused = solve_stats(torch, base, B)
        s, st = setup(m0)
        fresh = solve_stats(torch, s, B)
        fresh["setup_s"] = st
        s.close()
        mass.append(dict(shift=sh, m0=m0, reused=reused, fresh=fresh))
        _log("scans: m_crit + %g: reused outer %s TTS %.4fs | fresh outer %s TTS %.4fs setup %.3fs" %
             (sh, reused["outer_iters"], reused["time_to_solution_s"], fresh["outer_iters"],
              fresh["time_to_solution_s"], st))
    base.close()
    out["mass_scan"] = dict(setup_shift=0.02, setup_s=base_setup, points=mass)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
