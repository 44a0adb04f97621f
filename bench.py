#!/usr/bin/env python3
"""DD-alpha-AMG time-to-solution on one MI355X.

Workload (default): the 16^4 clover-Wilson system with links exp(i 0.4 H)
reunitarised to SU(3) and smeared by two APE steps (alpha 0.5, seed 0),
csw = 1, m0 = m_crit + 0.02 (m_crit of this field, estimated by Arnoldi on
the CPU oracle and stored in tests/golden/mcrit.json); two levels, aggregates
and SAP blocks 4^4, 3 MR steps, N = 20 test vectors, n_inv = 6, FP64
throughout; one complex N(0,1) right-hand side per solve; FGMRES(25) to a
true relative residual of 1e-10.

One step = one complete solve on the resident setup (the setup time is
reported separately).  Prints one JSON line with the time-to-solution, the
roofline figure of the dominant kernel (algorithmic bytes / live HIP-event
duration, accumulated by the library over the timed solves) and the CPU
oracle's time on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-kernels] [--no-variants] [--sched FLAGS]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_digest(path):
    import hashlib

    with open(os.path.join(ROOT, path), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def counter_traffic(kernel_class):
    """HBM bytes per launch of the kernel class from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE record of this workload, scaled by the plain-copy
    factors stored with it; None when no record exists or the kernel's source
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "counters_16x4_fp64_solve.json")
    if not os.path.exists(path):
        return None, "no counter record"
    with open(path) as f:
        rec = json.load(f)
    k = rec.get("kernels", {}).get(kernel_class)
    if not k:
        return None, "no counters for this kernel"
    if kernel_source_digest(k["source"]) != k["source_sha256"]:
        return None, "kernel changed since the counters were taken"
    by = (k["fetch_kib"] * rec["fetch_scale"] + k["write_kib"] * rec["write_scale"]) * 1024.0
    return by, "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, mean over %d dispatches" % k["dispatches"]


def load_mcrit(name):
    with open(os.path.join(ROOT, "tests", "golden", "mcrit.json")) as f:
        return json.load(f)[name]


def c2_problem():
    from paper_1303_1377_amd import fields as F

    info = load_mcrit("lat16x4_ape2_seed0")
    dims = tuple(info["dims"])
    U = F.make_gauge(dims, info["eps"], info["seed"], ape_steps=info["ape"], ape_alpha=0.5)
    m0 = info["m_crit"] + 0.02
    return dims, U, m0, info["csw"], info


def c2_params(G, **over):
    kw = dict(levels=2, n_tv=[20], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], mr_steps=[3], nu=2, n_inv=6,
              coarse_tol=5e-2, coarse_restart=30, outer_restart=25, precision=64)
    kw.update(over)
    return G.default_params(**kw), kw


def cpu_baseline(dims, U, m0, csw, kw, gpu_stats, budget_s=30.0):
    """Oracle (FP64 C, OpenMP) on a bounded sample of the same solve: P and
    D_c built once from random test vectors (untimed), then V-cycles with the
    GPU run's mean coarse-iteration count plus the outer D applies, timed and
    scaled by the GPU's outer-iteration count to one solve."""
    import numpy as np

    import oracle as O
    from paper_1303_1377_amd import fields as F

    vol = int(np.prod(dims))
    o = O.Oracle(dims, U, m0, csw)
    its = max(1, gpu_stats["outer_iters"])
    cfix = max(1, int(round(gpu_stats["coarse_iters"][1] / its)))
    okw = {k: v for k, v in kw.items() if k != "precision"}
    okw["coarse_fixed"] = cfix
    o.configure(**okw)
    o.set_vectors(0, F.random_vectors(vol, 12, kw["n_tv"][0], 77))
    o.build(0)
    o.mark_setup()
    r = F.gaussian_spinor(dims, 4242).reshape(-1)
    t0 = time.time()
    n = 0
    while True:
        z = o.vcycle(0, r)
        o.apply(z)
        n += 1
        if time.time() - t0 > budget_s / 2 or n >= 3:
            break
    per_it = (time.time() - t0) / n
    return dict(value=per_it * its, unit="s", cores=O.num_threads(), kind="oracle",
                sample="%d V-cycle(s) (coarse GMRES fixed at %d its) + outer D apply on the 16^4 problem, "
                       "P/D_c from random vectors; scaled by the GPU outer iteration count %d" % (n, cfix, its),
                seconds_per_outer_iteration=per_it)


def kernel_measurements(G, F):
    """Standalone stencil and SAP timings at 32^3 x 64 (working set above the
    256 MB last-level cache), FP64 and FP32."""
    import numpy as np

    dims = (64, 32, 32, 32)
    vol = int(np.prod(dims))
    t = time.time()
    rng_seed = 0
    U = F.make_gauge(dims, 0.4, rng_seed)
    log("bench: 32^3x64 links generated in %.1fs" % (time.time() - t))
    s = G.Solver(dims, U, -0.05, 1.0)
    del U
    out = {}
    ms = s.time_kernel("dirac64", reps=20)
    out["dirac_fp64_32c64"] = dict(ms=ms, GBs=vol * 192 * 8 / ms / 1e6, bytes_per_site=1536)
    for prec in (32, 64):
        s.configure(G.default_params(levels=2, n_tv=[20], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], mr_steps=[4],
                                     precision=prec))
        sz = 4 if prec == 32 else 8
        ms = s.time_kernel("dirac_prec", reps=20)
        out["dirac_fp%d_32c64" % prec] = dict(ms=ms, GBs=vol * 192 * sz / ms / 1e6, bytes_per_site=192 * sz)
        ms = s.time_kernel("sap", reps=5)
        out["sap_sweep_fp%d_32c64" % prec] = dict(ms=ms, GBs=vol * 216 * sz / ms / 1e6, bytes_per_site=216 * sz,
                                                   mr_steps=4)
        log("bench: kernels fp%d done" % prec)
    s.close()
    return out


def variants(G, F, dims, U, m0, csw, n_solves=3):
    """Same 16^4 problem in the other forms the library offers: FP32 and
    FP16-storage preconditioners (FP64 outer), and 12 right-hand sides solved
    as one batch; each with its own setup, timed over whole solves."""
    import numpy as np
    import torch

    out = {}
    rhs = [torch.as_tensor(F.gaussian_spinor(dims, 2000 + i)).to("cuda") for i in range(12)]
    for name, over in (("fp32_preconditioner", dict(precision=32)), ("fp16_storage_preconditioner", dict(precision=16)),
                       ("fp64_batch12", dict(max_rhs=12)), ("fp32_batch12", dict(precision=32, max_rhs=12))):
        s = G.Solver(dims, U, m0, csw)
        params, _ = c2_params(G, **over)
        t0 = time.time()
        s.setup(params=params)
        torch.cuda.synchronize()
        setup_s = time.time() - t0
        s.autotune(reps=5)
        if "batch" in name:
            B = torch.stack(rhs)
            s.solve_batch(B, 1e-10)  # warm-up (graph capture)
            torch.cuda.synchronize()
            t0 = time.time()
            X, st = s.solve_batch(B, 1e-10)
            torch.cuda.synchronize()
            el = time.time() - t0
            worst = max(x["true_relres"] for x in st)
            out[name] = dict(setup_s=setup_s, batch_s=el, solves_per_s=12 / el, rhs=12, true_relres_max=worst,
                             outer_iters=[x["outer_iters"] for x in st])
        else:
            s.solve(rhs[0], 1e-10)
            torch.cuda.synchronize()
            t0 = time.time()
            sts = [s.solve(rhs[1 + i], 1e-10)[1] for i in range(n_solves)]
            torch.cuda.synchronize()
            el = (time.time() - t0) / n_solves
            out[name] = dict(setup_s=setup_s, time_to_solution_s=el, solves_per_s=1 / el,
                             true_relres_max=max(x["true_relres"] for x in sts),
                             outer_iters=[x["outer_iters"] for x in sts])
        log("bench: variant %s %s" % (name, out[name]))
        s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernels", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--sched", type=int, default=None, help="launch schedule flags instead of the autotuned one")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1303_1377_amd as G
    from paper_1303_1377_amd import fields as F

    log("bench: generating the 16^4 field")
    dims, U, m0, csw, info = c2_problem()
    s = G.Solver(dims, U, m0, csw)
    params, kw = c2_params(G)
    torch.cuda.synchronize()
    t0 = time.time()
    s.setup(params=params)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    log("bench: setup %.3fs" % setup_s)
    coarse_tune = None
    if args.sched is None:
        sched, tune_ms = s.autotune(reps=5)
        log("bench: autotuned schedule %d (ms per schedule %s)" % (sched, ["%.3f" % t for t in tune_ms]))
        grid, ctimes = s.autotune_coarse(reps=3)
        sched = s.get_schedule()
        coarse_tune = dict(chosen_grid=grid, graph_replay=bool(sched & 16), ms_single_launches=ctimes[0],
                           ms_graph_replay=ctimes[1],
                           ms_cooperative={str(g): t for g, t in zip((16, 32, 64, 128), ctimes[2:6])},
                           ms_outer_solve={"single_launches": ctimes[6], "graph_replay": ctimes[7]})
        log("bench: coarse solver %s" % coarse_tune)
    else:
        s.set_schedule(args.sched)
        sched = args.sched
    rhs = [torch.as_tensor(F.gaussian_spinor(dims, 1000 + i)).to("cuda") for i in range(args.warmup + args.steps)]
    for i in range(args.warmup):
        s.solve(rhs[i], 1e-10)
    log("bench: warmup done")
    # live HIP-event timing inside the timed region of the classes that bracket
    # one launch each (a few dozen launches per solve); "coarse", "reduce",
    # "blas" and "coarse_step" bracket groups of launches and are timed on one
    # more solve after the timed region, so their events do not slow the solves
    single = ("sap", "dirac64", "dirac_prec", "restrict", "prolong", "coarse_sap")
    s.profile(True, classes=single)
    torch.cuda.synchronize()
    t0 = time.time()
    stats = []
    for i in range(args.steps):
        x, st = s.solve(rhs[args.warmup + i], 1e-10)
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.time() - t0
    prof = s.profile_read()
    s.profile(True)
    s.solve(rhs[args.warmup], 1e-10)
    prof_all = s.profile_read()
    s.profile(False)
    log("bench: timed %d solves in %.3fs" % (args.steps, elapsed))
    tts = elapsed / args.steps
    worst = max(st["true_relres"] for st in stats)
    assert all(st["converged"] for st in stats) and worst <= 1e-10, stats

    # dominant single-kernel class by time
    dom = max(single, key=lambda k: prof[k][1])
    n_l, ms_l, by_l = prof[dom]
    avg_ms = ms_l / max(n_l, 1)
    achieved = (by_l / max(n_l, 1)) / (avg_ms * 1e-3) / 1e9 if n_l else 0.0
    traffic, traffic_src = counter_traffic(dom)
    kernels = {k: dict(launches=v[0], total_ms=round(v[1], 3),
                       GBs=round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None) for k, v in prof_all.items()}

    out = dict(
        metric="DD-alphaAMG time-to-solution @relres 1e-10",
        value=tts,
        unit="s",
        n_gpus=1,
        steps=args.steps,
        warmup=args.warmup,
        ms_per_step=tts * 1e3,
        higher_is_better=False,
        scaling="weak",
        vs_baseline=None,
        dtype="f64",
        data="synthetic",
        config=dict(workload="16^4 clover-Wilson, 2-level FP64 DD-alphaAMG (APE-smeared exp(i0.4H) links, "
                             "m0=m_crit+0.02), 1 Gaussian RHS, FGMRES(25) to 1e-10",
                    dims=list(dims), m0=m0, m_crit=info["m_crit"], csw=csw, n_tv=20, aggregates="4^4",
                    sap_blocks="4^4", mr_steps=3, nu=2, n_inv=6, coarse="odd-even GMRES(30) to 5e-2"),
        setup_s=setup_s,
        solves_per_s=1.0 / tts,
        schedule=sched,
        coarse_solver_tuning=coarse_tune,
        outer_iters=[st["outer_iters"] for st in stats],
        coarse_iters_per_solve=[st["coarse_iters"][1] for st in stats],
        true_relres_max=worst,
        roofline=dict(bound="hbm", kernel=dom, achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=achieved / HBM_PEAK_GBS, traffic=traffic, traffic_source=traffic_src,
                      algorithmic_bytes_per_launch=(by_l / max(n_l, 1)), launches=n_l, avg_launch_ms=avg_ms),
        kernel_classes=kernels,
        kernel_classes_note="every class timed with HIP events over one extra solve after the timed region",
    )
    if not args.no_variants:
        try:
            out["variants_16x4"] = variants(G, F, dims, U, m0, csw)
        except Exception as e:  # measurement extras never hide the main line
            out["variants_16x4"] = dict(error=str(e))
    if not args.no_kernels:
        try:
            out["kernels_32c64"] = kernel_measurements(G, F)
        except Exception as e:  # measurement extras never hide the main line
            out["kernels_32c64"] = dict(error=str(e))
    if not args.no_cpu_baseline:
        log("bench: CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(dims, U, m0, csw, kw, stats[0])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
