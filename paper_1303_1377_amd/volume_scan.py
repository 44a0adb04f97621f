"""Synthetic replica of the paper's volume scan (Sec. 6, Table 7): iteration
count and time against the lattice volume at fixed parameters, with the
comparison solver beside DD-alpha-AMG on the same fields.

    python -m paper_1303_1377_amd.volume_scan [--lattices 48x16,48x24,48x32] [--solves 2]

Lattices T x L^3 with T = 48 (the paper's 48 x 16^3, 48 x 24^3, 48 x 32^3);
links exp(i 0.4 H) reunitarised to SU(3), two APE steps (alpha 0.5), seed 0,
drawn on the GPU (fields.make_gauge_device); csw 1; one bare mass for all
volumes, m0 = m_crit(16^4) + 0.02 = -0.0484 (the critical masses of these
fields differ by about 2e-4).  DD-alpha-AMG: two levels, aggregates and SAP
blocks 4^4, N = 20, 4 MR steps, nu = 2, n_inv = 6, coarsest odd-even
GMRES(30) to 5e-2, V-cycle in FP32, outer FGMRES(25) in FP64 to 1e-10 (the
paper's setting).  Comparison: FGMRES(25) preconditioned by 50 FP32 odd-even
BiCGStab steps (the paper's BiCGStab).  Gaussian right-hand sides.
Prints one JSON line.
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


def params(G):
    return G.default_params(levels=2, n_tv=[20], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], mr_steps=[4], nu=2,
                            n_inv=6, coarse_tol=5e-2, coarse_restart=30, outer_restart=25, precision=32)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--lattices", default="48x16,48x24,48x32")
    ap.add_argument("--solves", type=int, default=2)
    ap.add_argument("--no-bicgstab", action="store_true")
    a = ap.parse_args()

    import torch

    import paper_1303_1377_amd as G
    from paper_1303_1377_amd import fields as F

    with open(os.path.join(ROOT, "tests", "golden", "mcrit.json")) as f:
        m_crit = json.load(f)["lat16x4_ape2_seed0"]["m_crit"]
    m0 = m_crit + 0.02
    rows = []
    for lat in a.lattices.split(","):
        t_, l_ = (int(v) for v in lat.split("x"))
        dims = (t_, l_, l_, l_)
        U = F.make_gauge_device(dims, 0.4, 0, ape_steps=2, ape_alpha=0.5)
        s = G.Solver(dims, U, m0, 1.0)
        torch.cuda.synchronize()
        t = time.time()
        s.setup(params=params(G))
        torch.cuda.synchronize()
        setup_s = time.time() - t
        s.autotune(reps=2)
        s.autotune_coarse(reps=1)
        B = [torch.as_tensor(F.gaussian_spinor(dims, 4000 + i)).to("cuda") for i in range(a.solves)]
        dd = []
        for b in B:
            torch.cuda.synchronize()
            t = time.time()
            x, st = s.solve(b, 1e-10)
            torch.cuda.synchronize()
            dd.append((time.time() - t, st["outer_iters"], st["coarse_iters"][1], st["true_relres"]))
        row = dict(dims=list(dims), sites=t_ * l_ ** 3, setup_s=setup_s,
                   dd_time_to_solution_s=min(d[0] for d in dd), dd_outer_iters=[d[1] for d in dd],
                   dd_coarse_iters=[d[2] for d in dd], dd_true_relres_max=max(d[3] for d in dd))
        if not a.no_bicgstab:
            bi = []
            for b in B[:1]:
                torch.cuda.synchronize()
                t = time.time()
                x, st = s.solve_bicgstab(b, 1e-10, steps=50, precision=32)
                torch.cuda.synchronize()
                bi.append((time.time() - t, st["outer_iters"], st["coarse_iters"][0], st["true_relres"]))
            row.update(bicgstab_time_to_solution_s=bi[0][0], bicgstab_outer_iters=bi[0][1],
                       bicgstab_steps=bi[0][2], bicgstab_true_relres=bi[0][3],
                       speedup_solve=bi[0][0] / row["dd_time_to_solution_s"],
                       speedup_setup_plus_solve=bi[0][0] / (setup_s + row["dd_time_to_solution_s"]))
        _log("volume_scan: %s %s" % (lat, row))
        rows.append(row)
        s.close()
        del U
        torch.cuda.empty_cache()
    print(json.dumps(dict(m0=m0, m_crit_16x4=m_crit, rows=rows)), flush=True)


if __name__ == "__main__":
    main()
