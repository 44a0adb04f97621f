#!/usr/bin/env python3
"""DD-alpha-AMG time-to-solution on one MI355X.

Workload (default): twelve point sources on the 48^3 x 96 clover-Wilson
system.  Links exp(i 0.4 H) reunitarised to SU(3) and smeared by two APE steps
(alpha 0.5), seed 0, drawn on the GPU (fields.make_gauge_device); csw = 1;
m0 = m_crit + 0.005 with m_crit the critical mass of this field
(paper_1303_1377_amd/mcrit_fields.json).  Three levels: aggregates 4^4 then
2^4, N = 20 / 20, SAP blocks 4^4 / 2^4, 4 MR steps, nu = 2, n_inv = 6,
intermediate FGMRES(10) and coarsest odd-even GMRES(30) to 5e-2; the
preconditioner in FP32 (on the coarse levels the multi-right-hand-side stencil
runs on the matrix cores), the outer FGMRES(5) in FP64 to a true relative
residual of 1e-10.  The sources are the unit vectors at the origin for every
spin and colour, solved by dd_solve_batch in batches of four (the largest
batch whose FP64 outer Krylov workspace fits in HBM beside the setup).

One step = one batched solve of four point sources on the resident setup;
three steps solve all twelve (step i takes spin-colour indices 4(i mod 3) ..
4(i mod 3) + 3).  The setup is timed separately.  Prints one JSON line with the
time per step, the roofline figure of the dominant kernel class (algorithmic
bytes per launch over the mean launch duration, HIP events on the library's
stream around every launch of that class inside the timed region) and the CPU
oracle's time on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-extras] [--sched FLAGS] [--precision 32|16|64]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
C4 = dict(dims=(96, 48, 48, 48), eps=0.4, ape=2, seed=0, shift=0.005, key="lat96x48c3_ape2_seed0_dev")
CLASSES_ONE_KERNEL = ("dirac64", "dirac_prec", "sap", "restrict", "prolong", "coarse_sap")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_digest(path):
    import hashlib

    with open(os.path.join(ROOT, path), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def counter_traffic(record, kernel_class):
    """HBM bytes per launch of a kernel class from a committed rocprofv3
    FETCH_SIZE / WRITE_SIZE record (profiles/), scaled by the plain-copy
    factors stored with it; None when no record exists or the kernel's source
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", record)
    if not os.path.exists(path):
        return None, "no counter record"
    with open(path) as f:
        rec = json.load(f)
    k = rec.get("kernels", {}).get(kernel_class)
    if not k:
        return None, "no counters for this kernel class"
    if kernel_source_digest(k["source"]) != k["source_sha256"]:
        return None, "kernel source changed since the counters were taken"
    by = (k["fetch_kib"] * rec["fetch_scale"] + k["write_kib"] * rec["write_scale"]) * 1024.0
    return by, "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, mean over %d dispatches (%s)" % (k["dispatches"], record)


def load_mcrit(key):
    with open(os.path.join(ROOT, "paper_1303_1377_amd", "mcrit_fields.json")) as f:
        data = json.load(f)
    if key not in data:
        raise SystemExit("bench.py: no critical mass stored for %s (run python -m paper_1303_1377_amd.mcrit)" % key)
    return data[key]


def c4_params(G, precision, max_rhs):
    return G.default_params(levels=3, n_tv=[20, 20], agg=[(4, 4, 4, 4), (2, 2, 2, 2)],
                            sap=[(4, 4, 4, 4), (2, 2, 2, 2)], mr_steps=[4, 4], nu=2, n_inv=6, coarse_tol=5e-2,
                            coarse_restart=30, mid_tol=5e-2, mid_restart=10, outer_restart=5, precision=precision,
                            max_rhs=max_rhs)


def point_sources(torch, vol, first, count):
    """Unit vectors at site 0 for spin-colour indices first .. first+count-1 (3 spin + colour)."""
    b = torch.zeros((count, vol, 4, 3), dtype=torch.complex128, device="cuda")
    for q in range(count):
        sc = (first + q) % 12
        b[q, 0, sc // 3, sc % 3] = 1.0
    return b


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(dims, U, m0, step_stats, k, nu=2, mr=4):
    """The oracle (FP64 C, OpenMP on the host cores) on a bounded sample of the
    same workload: one D apply and one SAP sweep (4^4 blocks, 4 MR steps) on
    the full 48^3 x 96 lattice, timed.  Scaled to one step as
    k sources x outer iterations x (D apply + nu SAP sweeps): the fine-level
    work alone, so a lower bound of the oracle's time per step (the coarse
    levels, the transfers and the orthogonalisation are not included)."""
    import numpy as np

    import oracle as O
    from paper_1303_1377_amd import fields as F

    t0 = time.time()
    o = O.Oracle(dims, U, m0, 1.0)
    create_s = time.time() - t0
    o.configure(levels=2, n_tv=[1], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], mr_steps=[mr])
    b = F.gaussian_spinor(dims, 4242)
    t0 = time.time()
    o.apply(b)
    d_s = time.time() - t0
    t0 = time.time()
    o.sap(0, b, 1)
    sap_s = time.time() - t0
    o.close()
    its = float(np.mean([st["outer_iters"] for st in step_stats]))
    per_it = d_s + nu * sap_s
    return dict(value=k * its * per_it, unit="s", cores=O.num_threads(), kind="oracle",
                cpu_model=cpu_model(),
                sample="oracle on the full 48^3x96 lattice: 1 FP64 D apply (%.2f s) + 1 SAP sweep with 4 MR steps "
                       "(%.2f s), timed; scaled to one step as %d sources x %.1f outer iterations x (D + %d SAP "
                       "sweeps): fine level only, a lower bound (coarse levels, transfers and Gram-Schmidt "
                       "excluded); oracle context creation (clover) took %.1f s, untimed" %
                       (d_s, sap_s, k, its, nu, create_s),
                lower_bound=True, d_apply_s=d_s, sap_sweep_s=sap_s)


def extras_16x4(G, F):
    """The 16^4 problem of the two-level FP64 configuration (APE field, m0 =
    m_crit + 0.02, N = 20, 3 MR steps): time to solution of single solves."""
    import torch

    with open(os.path.join(ROOT, "tests", "golden", "mcrit.json")) as f:
        info = json.load(f)["lat16x4_ape2_seed0"]
    dims = tuple(info["dims"])
    U = F.make_gauge(dims, info["eps"], info["seed"], ape_steps=info["ape"], ape_alpha=0.5)
    m0 = info["m_crit"] + 0.02
    s = G.Solver(dims, U, m0, 1.0)
    t0 = time.time()
    s.setup(params=G.default_params(levels=2, n_tv=[20], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], mr_steps=[3],
                                    nu=2, n_inv=6, outer_restart=25, precision=64))
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    s.autotune(reps=3)
    s.autotune_coarse(reps=2)
    rhs = [torch.as_tensor(F.gaussian_spinor(dims, 1000 + i)).to("cuda") for i in range(6)]
    s.solve(rhs[0], 1e-10)
    torch.cuda.synchronize()
    t0 = time.time()
    sts = [s.solve(r, 1e-10)[1] for r in rhs[1:]]
    torch.cuda.synchronize()
    tts = (time.time() - t0) / 5
    s.close()
    return dict(workload="16^4, 2 levels, FP64, 1 Gaussian RHS", setup_s=setup_s, time_to_solution_s=tts,
                outer_iters=[x["outer_iters"] for x in sts], true_relres_max=max(x["true_relres"] for x in sts))


def extras_kernels_32c64(G, F):
    """Standalone stencil and SAP timings at 32^3 x 64 (device-drawn field,
    working set above the 256 MB last-level cache), FP64 and FP32, with the
    algorithmic bytes of the measurement tables (stencil 192 reals per site,
    SAP sweep 288 reals per site)."""
    dims = (64, 32, 32, 32)
    vol = 64 * 32 ** 3
    U = F.make_gauge_device(dims, 0.4, 0)
    s = G.Solver(dims, U, -0.05, 1.0)
    del U
    out = {}
    ms = s.time_kernel("dirac64", reps=20)
    out["dirac_fp64"] = dict(ms=ms, GBs=vol * 192 * 8 / ms / 1e6)
    for prec in (32, 64):
        s.configure(G.default_params(levels=2, n_tv=[20], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], mr_steps=[4],
                                     precision=prec))
        sz = 4 if prec == 32 else 8
        ms = s.time_kernel("dirac_prec", reps=20)
        out["dirac_fp%d" % prec] = dict(ms=ms, GBs=vol * 192 * sz / ms / 1e6)
        ms = s.time_kernel("sap", reps=5)
        out["sap_sweep_fp%d" % prec] = dict(ms=ms, GBs=vol * 288 * sz / ms / 1e6, mr_steps=4)
    s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--precision", type=int, default=32)
    ap.add_argument("--max-rhs", type=int, default=4)
    ap.add_argument("--sched", type=int, default=None, help="launch schedule flags instead of the autotuned ones")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (there is no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1303_1377_amd as G
    from paper_1303_1377_amd import fields as F

    dims = C4["dims"]
    vol = int(np.prod(dims))
    mc = load_mcrit(C4["key"])
    m0 = mc["m_crit"] + C4["shift"]
    t0 = time.time()
    U = F.make_gauge_device(dims, C4["eps"], C4["seed"], ape_steps=C4["ape"], ape_alpha=0.5)
    torch.cuda.synchronize()
    field_s = time.time() - t0
    U_host = None if args.no_cpu_baseline else U.cpu().numpy()
    log("bench: 48^3x96 field in %.1fs, m_crit %.6f, m0 %.6f" % (field_s, mc["m_crit"], m0))
    s = G.Solver(dims, U, m0, 1.0)
    k = args.max_rhs
    params = c4_params(G, args.precision, k)
    torch.cuda.synchronize()
    t0 = time.time()
    s.setup(params=params)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    log("bench: setup %.1fs, %.1f GB on the device" % (setup_s, s.device_bytes() / 1e9))
    tuning = None
    if args.sched is None:
        sched, tune_ms = s.autotune(reps=2)
        grid, ctimes = s.autotune_coarse(reps=1)
        tuning = dict(fine_schedule=sched, fine_ms=tune_ms, coarse_grid=grid, coarse_ms=ctimes,
                      schedule=s.get_schedule())
        log("bench: tuning %s" % tuning)
    else:
        s.set_schedule(args.sched)

    def step(i):
        b = point_sources(torch, vol, 4 * (i % 3), k)
        x, st = s.solve_batch(b, 1e-10)
        return st

    for i in range(args.warmup):
        step(i)
    # one more step, untimed, with every kernel class timed: finds the dominant class
    s.profile(True)
    step(0)
    prof_all = s.profile_read()
    s.profile(False)
    dom = max(CLASSES_ONE_KERNEL, key=lambda c: prof_all[c][1])
    dom_any = max(prof_all, key=lambda c: prof_all[c][1])
    log("bench: warmup done; dominant single-kernel class %s (largest class of any kind: %s)" % (dom, dom_any))
    # timed region: events only around the launches of the dominant class
    s.profile(True, classes=(dom,))
    torch.cuda.synchronize()
    t0 = time.time()
    stats = []
    for i in range(args.steps):
        stats += step(i)
    torch.cuda.synchronize()
    elapsed = time.time() - t0
    prof = s.profile_read()
    s.profile(False)
    per_step = elapsed / args.steps
    worst = max(st["true_relres"] for st in stats)
    log("bench: timed %d steps in %.2fs (%.3f s per step of %d sources)" % (args.steps, elapsed, per_step, k))
    assert all(st["converged"] for st in stats) and worst <= 1e-10, stats
    n_l, ms_l, by_l = prof[dom]
    avg_ms = ms_l / max(n_l, 1)
    per_launch = by_l / max(n_l, 1)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if n_l else 0.0
    traffic, traffic_src = counter_traffic("counters_48c96_fp32_batch4.json", dom)
    kernels = {c: dict(launches=v[0], total_ms=round(v[1], 2),
                       GBs=round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None) for c, v in prof_all.items()}
    s.close()
    del U
    torch.cuda.empty_cache()

    out = dict(
        metric="DD-alphaAMG time-to-solution @relres 1e-10",
        value=per_step,
        unit="s",
        n_gpus=1,
        steps=args.steps,
        warmup=args.warmup,
        ms_per_step=per_step * 1e3,
        higher_is_better=False,
        scaling="weak",
        vs_baseline=None,
        dtype="f32" if args.precision == 32 else ("f16-storage/f32" if args.precision == 16 else "f64"),
        data="synthetic",
        config=dict(workload="48^3x96 clover-Wilson, 12 point sources (origin, every spin-colour) in batches of %d; "
                             "3-level DD-alphaAMG, FP%d preconditioner, FP64 outer FGMRES(5) to 1e-10; "
                             "one step = one batch" % (k, args.precision),
                    dims=list(dims), m0=m0, m_crit=mc["m_crit"], m_crit_method=mc["method"], csw=1.0,
                    field="exp(i0.4H) SU(3), 2 APE steps (alpha 0.5), seed 0, drawn on the GPU",
                    n_tv=[20, 20], aggregates=["4^4", "2^4"], sap_blocks=["4^4", "2^4"], mr_steps=4, nu=2, n_inv=6,
                    coarse="odd-even GMRES(30) to 5e-2", intermediate="FGMRES(10) to 5e-2",
                    rhs_per_step=k, precision=args.precision),
        seconds_per_12_sources=per_step * 12.0 / k,
        solves_per_s=k / per_step,
        setup_s=setup_s,
        field_s=field_s,
        tuning=tuning,
        outer_iters=[st["outer_iters"] for st in stats],
        coarse_iters=[list(st["coarse_iters"][:3]) for st in stats],
        true_relres_max=worst,
        roofline=dict(bound="hbm", kernel=dom, achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=achieved / HBM_PEAK_GBS, traffic=traffic, traffic_source=traffic_src,
                      algorithmic_bytes_per_launch=per_launch, launches=n_l, avg_launch_ms=avg_ms),
        kernel_classes=kernels,
        kernel_classes_note="every class timed with HIP events over one untimed step before the timed region; "
                            "the largest class of any kind was %s" % dom_any,
    )
    if not args.no_extras:
        for name, fn in (("extra_16x4_fp64", extras_16x4), ("extra_kernels_64x32c3", extras_kernels_32c64)):
            try:
                t = time.time()
                out[name] = fn(G, F)
                log("bench: %s in %.1fs: %s" % (name, time.time() - t, out[name]))
            except Exception as e:  # extras never hide the main line
                out[name] = dict(error=str(e))
            torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("bench: CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(dims, U_host, m0, stats, k)
        del U_host
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
