"""Twelve point sources (unit vector at the origin for every spin and colour)
solved batched on a large lattice, against the plain FP64 one-at-a-time form.

    python -m paper_1303_1377_amd.batched_sources [--dims 96,48,48,48]
        [--max-rhs 4] [--precision 32] [--outer-restart 5] [--baseline-rhs 2]
        [--shift 0.005] [--tol 1e-10] [--levels 3|4]

Field: links exp(i 0.4 H) reunitarised to SU(3), two APE steps (alpha 0.5),
seed 0, drawn on the GPU (fields.make_gauge_device: the host recipe, a
different random stream); csw 1; m0 = m_crit + shift with m_crit of this
field (paper_1303_1377_amd/mcrit_fields.json).  Hierarchy: three levels,
aggregates 4^4 then 2^4, N = 20 / 20, SAP blocks 4^4 and 2^4, 4 MR steps
(--levels 4: a further level, SAP blocks 2x3^3 on level 2 and a coarsest
6x3^3 lattice with plain GMRES); preconditioner in `precision`, FP64 outer
FGMRES(outer_restart) (a short restart length keeps the outer Krylov basis of
max_rhs right-hand sides in HBM).  The 12 sources run through dd_solve_batch
in batches of max_rhs: on the coarse levels with 2..16 FP32 right-hand sides
the stencil runs on the matrix cores, and the coarsest GMRES steps are
replayed as HIP graphs; the fine-kernel and coarse-solver schedules come from
the autotuners.  The baseline solves the first `baseline_rhs` sources one at a
time with an FP64 preconditioner (its own setup).  Prints one JSON line.
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


def params(G, precision, max_rhs, outer_restart, levels=3):
    if levels == 4:
        # level 2 of 96x48^3 is 12x6^3: SAP blocks 2x3^3 (an even block count per
        # direction), aggregates 2^4 onto a coarsest 6x3^3 (odd extent: plain GMRES)
        return G.default_params(levels=4, n_tv=[20, 20, 20], agg=[(4, 4, 4, 4), (2, 2, 2, 2), (2, 2, 2, 2)],
                                sap=[(4, 4, 4, 4), (2, 2, 2, 2), (2, 3, 3, 3)], mr_steps=[4, 4, 4],
                                precision=precision, max_rhs=max_rhs, outer_restart=outer_restart)
    return G.default_params(levels=3, n_tv=[20, 20], agg=[(4, 4, 4, 4), (2, 2, 2, 2)],
                            sap=[(4, 4, 4, 4), (2, 2, 2, 2)], mr_steps=[4, 4], precision=precision,
                            max_rhs=max_rhs, outer_restart=outer_restart)


def sources(torch, vol, first, count):
    """Point sources first .. first+count-1 (spin-colour index sc = 3 spin + colour) at site 0."""
    b = torch.zeros((count, vol, 4, 3), dtype=torch.complex128, device="cuda")
    for q in range(count):
        sc = first + q
        b[q, 0, sc // 3, sc % 3] = 1.0
    return b


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", default="96,48,48,48")
    ap.add_argument("--max-rhs", type=int, default=4)
    ap.add_argument("--precision", type=int, default=32)
    ap.add_argument("--outer-restart", type=int, default=5)
    ap.add_argument("--baseline-rhs", type=int, default=2)
    ap.add_argument("--shift", type=float, default=0.005)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--levels", type=int, default=3, choices=(3, 4))
    a = ap.parse_args()
    dims = tuple(int(v) for v in a.dims.split(","))

    import torch

    import paper_1303_1377_amd as G
    from paper_1303_1377_amd import fields as F
    from paper_1303_1377_amd.serving import estimate_bytes

    # the field's own critical mass where it is stored, else the 16^4 one
    with open(os.path.join(ROOT, "paper_1303_1377_amd", "mcrit_fields.json")) as f:
        mc = json.load(f)
    key = "lat%dx%dc3_ape2_seed0_dev" % (dims[0], dims[1])
    m_crit = mc[key]["m_crit"] if key in mc and dims[1] == dims[2] == dims[3] else mc["lat16x4_ape2_seed0"]["m_crit"]
    m0 = m_crit + a.shift
    vol = dims[0] * dims[1] * dims[2] * dims[3]
    t0 = time.time()
    U = F.make_gauge_device(dims, 0.4, 0, ape_steps=2, ape_alpha=0.5, log=_log)
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    _log("batched_sources: %s field in %.1fs" % ("x".join(map(str, dims)), gen_s))

    def run_form(precision, max_rhs, first, count, tune):
        p = params(G, precision, max_rhs, a.outer_restart, a.levels)
        est = estimate_bytes(dims, p, max_rhs)
        s = G.Solver(dims, U, m0, 1.0)
        torch.cuda.synchronize()
        t = time.time()
        s.setup(params=p)
        torch.cuda.synchronize()
        setup_s = time.time() - t
        _log("batched_sources: FP%d setup (max_rhs %d) in %.1fs, %.1f GB on the device (estimate %.1f GB)" %
             (precision, max_rhs, setup_s, s.device_bytes() / 1e9, est / 1e9))
        sched = coarse = None
        if tune:
            sched, _ = s.autotune(reps=2)
            grid, _ = s.autotune_coarse(reps=1)
            coarse = grid
            _log("batched_sources: schedule %d, coarse solver grid %d" % (sched, grid))
        stats, times, xs = [], [], []
        s.profile(True)
        for c0 in range(first, first + count, max_rhs):
            k = min(max_rhs, first + count - c0)
            b = sources(torch, vol, c0, k)
            torch.cuda.synchronize()
            t = time.time()
            x, st = s.solve_batch(b, a.tol) if max_rhs > 1 else s.solve(b[0], a.tol)
            torch.cuda.synchronize()
            times.append(time.time() - t)
            st = st if isinstance(st, list) else [st]
            stats += st
            xs.append(x.reshape(k, vol, 4, 3)[:, :: max(1, vol // 4096)].cpu())   # a sample of sites
            _log("batched_sources: FP%d sources %d..%d in %.2fs, outer %s, true residual %.2e" %
                 (precision, c0, c0 + k - 1, times[-1], [q["outer_iters"] for q in st],
                  max(q["true_relres"] for q in st)))
            del b, x
        prof = s.profile_read()
        s.profile(False)
        out = dict(precision=precision, max_rhs=max_rhs, setup_s=setup_s, device_bytes=s.device_bytes(),
                   estimated_bytes=est, schedule=sched, coarse_grid=coarse, solve_s=times,
                   solves_per_s=count / sum(times), outer_iters=[q["outer_iters"] for q in stats],
                   coarse_iters=[list(q["coarse_iters"][:a.levels]) for q in stats],
                   true_relres=[q["true_relres"] for q in stats],
                   kernel_classes_ms={k: dict(launches=v[0], ms=round(v[1], 2)) for k, v in prof.items() if v[0]})
        s.close()
        torch.cuda.empty_cache()
        return out, torch.cat(xs)

    batched, xb = run_form(a.precision, a.max_rhs, 0, 12, True)
    res = dict(metric="12 point sources, batched mixed-precision vs FP64 one at a time", dims=list(dims), m0=m0,
               levels=a.levels,
               m_crit_used=m_crit, shift=a.shift, tol=a.tol, outer_restart=a.outer_restart, field_seconds=gen_s,
               batched=batched)
    if a.baseline_rhs > 0:
        base, x64 = run_form(64, 1, 0, a.baseline_rhs, False)
        res["baseline_fp64_one_at_a_time"] = base
        d = xb[: a.baseline_rhs] - x64
        res["sampled_rel_diff_vs_fp64"] = float(torch.linalg.norm(d) / torch.linalg.norm(x64))
        res["batched_vs_baseline_solves_per_s"] = batched["solves_per_s"] / base["solves_per_s"]
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
