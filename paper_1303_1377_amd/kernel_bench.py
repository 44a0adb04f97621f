"""Standalone timing of the fine-level kernels on one lattice.

    python -m paper_1303_1377_amd.kernel_bench [--dims 64,32,32,32]
        [--kernels copy,dirac64,dirac32,sap32,sap64] [--reps 20] [--mr 4]
        [--sched 0,1,2,3] [--device-field]

Each kernel is launched `reps` times back to back between two HIP events on
internal random data (dd_time_kernel); one JSON line reports the mean launch
duration and the algorithmic bandwidth (bytes every launch must move, counted
once: see the byte model below).  The same command under rocprofv3 gives the
kernel trace and the memory counters of exactly these launches.

Byte model per lattice site (reals of the storage precision):
  stencil   192 = links 72 + clover 72 + spinor in 24 + spinor out 24
  SAP sweep 288 = links 72 + clover 72 + b 24 + z read 24 + z write 24 + the
            residual 24 + the face values of the neighbouring blocks 48 (each
            site is solved once per sweep, in the half sweep of its colour)
  copy      one FP64 spinor read and written: 2 x 24 reals of 8 bytes
  coarse    per coarse site: 9 blocks of nd x nd complex (storage precision)
            + k input and k output vectors of nd complex FP32; flops 9 nd^2 k x 8
            (kernel names coarse<precision>x<k>, e.g. coarse32x12, coarse16x12)
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def run(dims=(64, 32, 32, 32), kernels=("copy", "dirac64", "dirac32", "sap32", "sap64"), reps=20, mr=4, seed=0,
        scheds=(3,), device_field=False):
    import numpy as np

    import paper_1303_1377_amd as G
    from paper_1303_1377_amd import fields as F

    vol = int(np.prod(dims))
    t = time.time()
    U = F.make_gauge_device(dims, 0.4, seed) if device_field else F.make_gauge(dims, 0.4, seed)
    _log("kernel_bench: %s links in %.1fs" % ("x".join(map(str, dims)), time.time() - t))
    s = G.Solver(dims, U, -0.05, 1.0)
    del U
    out = {}
    configured = None
    for k, sc in [(k, sc) for k in kernels for sc in (scheds if k != "copy" else (None,))]:
        if sc is not None:
            s.set_schedule(sc)
        if k.startswith("coarse"):
            # coarse<prec>x<k>: D_c of level 1 (aggregates 4^4, N = 20) on k RHS at once
            prec_s, kk = k[len("coarse"):].split("x")
            prec, kk = int(prec_s), int(kk)
            if configured != ("coarse", prec, kk, sc):
                s.setup(params=G.default_params(levels=2, n_tv=[20], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)],
                                                mr_steps=[mr], precision=prec, n_inv=0, max_rhs=kk))
                if sc is not None:
                    s.set_schedule(sc)
                configured = ("coarse", prec, kk, sc)
            ms = s.time_kernel("coarse", reps=reps)
            vol_c, nd = s.level_size(1)
            sz = 8 if prec != 16 else 4
            by = vol_c * (9 * nd * nd * sz + 2 * kk * nd * 8)
            fl = vol_c * 9 * nd * nd * kk * 8
            key = k if sc is None or len(scheds) == 1 else "%s_sched%d" % (k, sc)
            out[key] = dict(ms=ms, GBs=by / (ms * 1e-3) / 1e9, bytes=by, TFLOPs=fl / (ms * 1e-3) / 1e12, sched=sc)
            _log("kernel_bench: %s %.4f ms %.0f GB/s %.1f TFLOP/s" % (key, ms, out[key]["GBs"], out[key]["TFLOPs"]))
            continue
        if k in ("copy", "dirac64"):
            ms = s.time_kernel("blas" if k == "copy" else "dirac64", reps=reps)
            by = vol * (2 * 24 * 8 if k == "copy" else 192 * 8)
        else:
            prec = 32 if k.endswith("32") else 64
            if configured != prec:
                s.configure(G.default_params(levels=2, n_tv=[20], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)],
                                             mr_steps=[mr], precision=prec))
                configured = prec
            sz = prec // 8
            if k.startswith("dirac"):
                ms = s.time_kernel("dirac_prec", reps=reps)
                by = vol * 192 * sz
            else:
                ms = s.time_kernel("sap", reps=reps)
                by = vol * 288 * sz
        key = k if sc is None or len(scheds) == 1 else "%s_sched%d" % (k, sc)
        out[key] = dict(ms=ms, GBs=by / (ms * 1e-3) / 1e9, bytes=by, sched=sc)
        _log("kernel_bench: %s %.4f ms %.0f GB/s" % (key, ms, out[key]["GBs"]))
    s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", default="64,32,32,32")
    ap.add_argument("--kernels", default="copy,dirac64,dirac32,sap32,sap64")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--mr", type=int, default=4)
    ap.add_argument("--sched", default="3", help="comma-separated launch schedules (DD_SCHED_* flag sets)")
    ap.add_argument("--device-field", action="store_true", help="draw the links on the GPU (large lattices)")
    a = ap.parse_args()
    dims = tuple(int(v) for v in a.dims.split(","))
    res = run(dims, tuple(a.kernels.split(",")), a.reps, a.mr, scheds=tuple(int(v) for v in a.sched.split(",")),
              device_field=a.device_field)
    print(json.dumps(dict(dims=list(dims), reps=a.reps, mr_steps=a.mr, kernels=res)), flush=True)


if __name__ == "__main__":
    main()
