"""Times of the FP64 CPU oracle on the benchmark configurations.

Measurement infrastructure beside the oracle (it runs the oracle only; the
GPU library is not loaded).  Prints one JSON object per configuration:

  4^4 (two levels, N = 8, aggregates and SAP blocks 2^4, m0 = -0.4):
      the whole setup (Algorithm 2, n_inv = 6) and a solve to 1e-10.
  16^4 (two levels, N = 20, 4^4, 3 MR steps, APE field, m_crit + 0.02):
      the whole setup and a solve to 1e-10.
  64x32^3 (three levels, 4^4 then 2^4, N = 20 / 20): one D apply, one SAP
      sweep (4 MR steps), one level-1 D_c apply, one restriction and one
      prolongation, and one V-cycle (coarse GMRES to 5e-2, middle FGMRES(10)
      to 5e-2) on P and D_c built from random test vectors.
  96x48^3: one D apply and one SAP sweep (the bench's CPU leg, at its size).

    python -m oracle.time_configs [--only 4x4,16x4,64x32c3,96x48c3]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _t(f, *a, **k):
    t0 = time.time()
    r = f(*a, **k)
    return time.time() - t0, r


def full_solve(name, dims, U, m0, kw, tol=1e-10, seed=1000):
    import oracle as O
    from paper_1303_1377_amd import fields as F

    o = O.Oracle(dims, U, m0, 1.0)
    o.configure(**kw)
    vol = int(np.prod(dims))
    setup_s, _ = _t(o.setup, [F.random_vectors(vol, 12, kw["n_tv"][0], 77)])
    b = F.gaussian_spinor(dims, seed)
    solve_s, (x, st) = _t(o.solve, b, tol)
    d_s, _ = _t(o.apply, b)
    sap_s, _ = _t(o.sap, 0, b, 1)
    o.close()
    return dict(config=name, dims=list(dims), setup_s=setup_s, solve_s=solve_s, total_s=setup_s + solve_s,
                outer_iters=st["outer_iters"], coarse_iters=st["coarse_iters"][:kw["levels"]],
                true_relres=st["true_relres"], d_apply_s=d_s, sap_sweep_s=sap_s)


def components(name, dims, U, m0, three_level=True, with_coarse=True):
    import oracle as O
    from paper_1303_1377_amd import fields as F

    out = dict(config=name, dims=list(dims))
    o = O.Oracle(dims, U, m0, 1.0)
    kw = dict(levels=3, n_tv=[20, 20], agg=[(4, 4, 4, 4), (2, 2, 2, 2)], sap=[(4, 4, 4, 4), (2, 2, 2, 2)],
              mr_steps=[4, 4]) if three_level else dict(levels=2, n_tv=[1], agg=[(4, 4, 4, 4)],
                                                        sap=[(4, 4, 4, 4)], mr_steps=[4])
    o.configure(**kw)
    b = F.gaussian_spinor(dims, 4242)
    out["d_apply_s"], _ = _t(o.apply, b)
    out["sap_sweep_s"], _ = _t(o.sap, 0, b, 1)
    if with_coarse:
        vol0, _ = o.level_size(0)
        o.set_vectors(0, F.random_vectors(vol0, 12, 20, 5))
        out["build_level0_s"], _ = _t(o.build, 0)
        vol1, nd1 = o.level_size(1)
        o.set_vectors(1, F.random_vectors(vol1, nd1, 20, 6))
        out["build_level1_s"], _ = _t(o.build, 1)
        o.mark_setup()
        rng = np.random.default_rng(7)
        vc = rng.standard_normal((vol1, nd1)) + 1j * rng.standard_normal((vol1, nd1))
        out["coarse_apply_level1_s"], _ = _t(o.apply, vc, 1)
        out["restrict_s"], _ = _t(o.restrict, 0, b)
        out["prolong_s"], _ = _t(o.prolong, 0, vc)
        out["vcycle_s"], _ = _t(o.vcycle, 0, b)
    o.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="4x4,16x4,64x32c3,96x48c3")
    a = ap.parse_args()
    import oracle as O
    from paper_1303_1377_amd import fields as F

    want = set(a.only.split(","))
    info = dict(cpu_model=_cpu_model(), threads=O.num_threads())
    print(json.dumps(info), flush=True)
    if "4x4" in want:
        dims = (4, 4, 4, 4)
        U = F.make_gauge(dims, 0.3, 0)
        kw = dict(levels=2, n_tv=[8], agg=[(2, 2, 2, 2)], sap=[(2, 2, 2, 2)], mr_steps=[4], n_inv=6,
                  outer_restart=20)
        print(json.dumps(full_solve("4^4", dims, U, -0.4, kw)), flush=True)
    if "16x4" in want:
        with open(os.path.join(ROOT, "tests", "golden", "mcrit.json")) as f:
            mc = json.load(f)["lat16x4_ape2_seed0"]
        dims = tuple(mc["dims"])
        U = F.make_gauge(dims, mc["eps"], mc["seed"], ape_steps=mc["ape"], ape_alpha=0.5)
        kw = dict(levels=2, n_tv=[20], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], mr_steps=[3], n_inv=6,
                  outer_restart=20)
        print(json.dumps(full_solve("16^4", dims, U, mc["m_crit"] + 0.02, kw)), flush=True)
    if "64x32c3" in want:
        dims = (64, 32, 32, 32)
        t0 = time.time()
        U = F.make_gauge(dims, 0.4, 0, ape_steps=2, ape_alpha=0.5)
        r = components("64x32^3", dims, U, -0.0585)
        r["field_s"] = time.time() - t0
        print(json.dumps(r), flush=True)
        del U
    if "96x48c3" in want:
        dims = (96, 48, 48, 48)
        t0 = time.time()
        U = F.make_gauge(dims, 0.4, 0, ape_steps=2, ape_alpha=0.5)
        r = components("96x48^3", dims, U, -0.0636, three_level=False, with_coarse=False)
        r["field_s"] = time.time() - t0
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
