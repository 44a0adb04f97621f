"""Three-level solves of one large system with the preconditioner in FP64,
FP32 and FP16 storage (FP32 arithmetic); the outer FGMRES is FP64 in all
three.  For each form: setup time, time to solution, iteration counts, the
true relative residual and the distance of the solution from the
FP64-preconditioned one.

    python -m paper_1303_1377_amd.precision_study [--dims 64,32,32,32]
        [--m0 M] [--mcrit-key lat64x32c3_ape2_seed0] [--precisions 64,32,16]
        [--solves 2] [--tol 1e-10] [--levels 3]

The field is the 32^3 x 64 workload: links exp(i 0.4 H) reunitarised to
SU(3), two APE steps (alpha 0.5), seed 0, csw 1, m0 = m_crit + 0.01 with
m_crit from tests/golden/mcrit.json when --m0 is not given.  Hierarchy:
aggregates 4^4 then 2^4 (with --levels 4 one more 2^4 level), N = 20
per level, SAP blocks 4^4 (fine) and 2^4 (coarse levels), 4 MR steps, nu = 2,
n_inv = 6; intermediate FGMRES(10) and
coarsest odd-even GMRES(30) to 5e-2; FGMRES(25) outer.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def params(G, precision, levels=3, **over):
    # levels 3: aggregates 4^4 then 2^4; levels 4: one more 2^4 level
    extra = levels - 2
    kw = dict(levels=levels, n_tv=[20] * (levels - 1), agg=[(4, 4, 4, 4)] + [(2, 2, 2, 2)] * extra,
              sap=[(4, 4, 4, 4)] + [(2, 2, 2, 2)] * extra, mr_steps=[4] * (levels - 1), nu=2, n_inv=6,
              coarse_tol=5e-2, coarse_restart=30, mid_tol=5e-2, mid_restart=10, outer_restart=25,
              precision=precision)
    kw.update(over)
    return G.default_params(**kw)


def run(dims, m0, precisions=(64, 32, 16), solves=2, tol=1e-10, seed=0, ape=2, n_inv=6, levels=3):
    import numpy as np
    import torch

    import paper_1303_1377_amd as G
    from paper_1303_1377_amd import fields as F

    t = time.time()
    U = F.make_gauge(dims, 0.4, seed, ape_steps=ape, ape_alpha=0.5)
    _log("precision_study: field %s in %.1fs" % ("x".join(map(str, dims)), time.time() - t))
    B = [torch.as_tensor(F.gaussian_spinor(dims, 7000 + i)).to("cuda") for i in range(solves)]
    res = {}
    ref = None
    for prec in precisions:
        s = G.Solver(dims, U, m0, 1.0)
        torch.cuda.synchronize()
        t0 = time.time()
        s.setup(params=params(G, prec, levels=levels, n_inv=n_inv))
        torch.cuda.synchronize()
        setup_s = time.time() - t0
        s.autotune(reps=3)
        s.autotune_coarse(reps=1)
        xs, sts, times = [], [], []
        for b in B:
            torch.cuda.synchronize()
            t0 = time.time()
            x, st = s.solve(b, tol)
            torch.cuda.synchronize()
            times.append(time.time() - t0)
            xs.append(x)
            sts.append(st)
        # time per kernel class over one more solve (live HIP events)
        s.profile(True)
        s.solve(B[0], tol)
        prof = s.profile_read()
        s.profile(False)
        classes = {k: dict(launches=v[0], ms=round(v[1], 3)) for k, v in prof.items() if v[0]}
        if ref is None and prec == 64:
            ref = xs
        dev = None
        if ref is not None:
            dev = max(float(torch.linalg.norm(x - r) / torch.linalg.norm(r)) for x, r in zip(xs, ref))
        res["fp%d" % prec if prec != 16 else "fp16_storage"] = dict(
            precision=prec, setup_s=setup_s, time_to_solution_s=float(np.median(times)), solve_s=times,
            outer_iters=[st["outer_iters"] for st in sts], coarse_iters=[list(st["coarse_iters"][:levels]) for st in sts],
            true_relres=[st["true_relres"] for st in sts], rel_diff_vs_fp64_form=dev, device_bytes=s.device_bytes(),
            schedule=s.get_schedule(), kernel_classes_ms=classes)
        _log("precision_study:", prec, res["fp%d" % prec if prec != 16 else "fp16_storage"])
        s.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", default="64,32,32,32")
    ap.add_argument("--m0", type=float, default=None)
    ap.add_argument("--mcrit-key", default="lat64x32c3_ape2_seed0")
    ap.add_argument("--shift", type=float, default=0.01)
    ap.add_argument("--precisions", default="64,32,16")
    ap.add_argument("--solves", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--n-inv", type=int, default=6)
    ap.add_argument("--levels", type=int, default=3)
    a = ap.parse_args()
    dims = tuple(int(v) for v in a.dims.split(","))
    if a.m0 is None:
        with open(os.path.join(ROOT, "tests", "golden", "mcrit.json")) as f:
            m_crit = json.load(f)[a.mcrit_key]["m_crit"]
        m0 = m_crit + a.shift
    else:
        m_crit, m0 = None, a.m0
    res = run(dims, m0, tuple(int(p) for p in a.precisions.split(",")), a.solves, a.tol, n_inv=a.n_inv,
              levels=a.levels)
    print(json.dumps(dict(dims=list(dims), m0=m0, m_crit=m_crit, tol=a.tol, levels=a.levels, forms=res)), flush=True)


if __name__ == "__main__":
    main()
