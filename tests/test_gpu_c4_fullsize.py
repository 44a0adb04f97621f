"""GPU parity at the full size of the benchmarked workload: 96x48^3, the
device-drawn APE field of the benchmark, m0 = m_crit + 0.005 of this field,
the benchmark's three-level FP32 hierarchy and batches of four right-hand
sides in one launch, with the schedule the autotuners pick.  The oracle runs
on the host on the same field (about 10 s to build its clover, 0.5 s per D
apply and 4 s per SAP sweep on 16 threads).

* FP64 stencil: every entry against the oracle, 1e-13 of the largest.
* FP32 SAP sweep (4^4 blocks, 4 MR steps) with four right-hand sides in one
  launch: each against the oracle's sweep, at the FP32 SAP bar of the small
  cases (1e-5).
* The benchmark's solve of four point sources: each true residual, with the
  oracle's D applied to the returned x, at most 1e-10, and the reported
  residual agreeing with it."""
import json
import os

import numpy as np
import pytest

from tests._gpu import rel, say, to_np

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DIMS = (96, 48, 48, 48)


def c4_params(G, precision=32, max_rhs=4):
    return G.default_params(levels=3, n_tv=[20, 20], agg=[(4, 4, 4, 4), (2, 2, 2, 2)],
                            sap=[(4, 4, 4, 4), (2, 2, 2, 2)], mr_steps=[4, 4], nu=2, n_inv=6, coarse_tol=5e-2,
                            coarse_restart=30, mid_tol=5e-2, mid_restart=10, outer_restart=5,
                            precision=precision, max_rhs=max_rhs)


@pytest.fixture(scope="module")
def c4():
    import torch

    import oracle as O
    import paper_1303_1377_amd as G
    from paper_1303_1377_amd import fields as F

    with open(os.path.join(ROOT, "paper_1303_1377_amd", "mcrit_fields.json")) as f:
        m0 = json.load(f)["lat96x48c3_ape2_seed0_dev"]["m_crit"] + 0.005
    say("case: 96x48^3 full size, device field, m0 = %.6f" % m0)
    U = F.make_gauge_device(DIMS, 0.4, 0, ape_steps=2, ape_alpha=0.5)
    torch.cuda.synchronize()
    o = O.Oracle(DIMS, U.cpu().numpy(), m0, 1.0)
    # the oracle's SAP needs only the fine level's blocks (no test vectors at this size)
    o.configure(levels=2, n_tv=[1], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], mr_steps=[4])
    s = G.Solver(DIMS, U, m0, 1.0)
    del U
    yield s, o, G, torch
    s.close()
    o.close()
    torch.cuda.empty_cache()


def _random(torch, k, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    vol = int(np.prod(DIMS))
    re = torch.randn((k, vol, 4, 3), generator=g, device="cuda", dtype=torch.float64)
    im = torch.randn((k, vol, 4, 3), generator=g, device="cuda", dtype=torch.float64)
    return torch.complex(re, im)


def test_c4_stencil_fp64(c4):
    s, o, G, torch = c4
    v = _random(torch, 1, 11)[0]
    y, _ = s.apply("D", 0, v)
    err = rel(to_np(y), o.apply(to_np(v)))
    say("  96x48^3 FP64 stencil: %.2e" % err)
    assert err < 1e-13


def test_c4_sap_fp32_four_rhs_in_one_launch(c4):
    s, o, G, torch = c4
    s.configure(c4_params(G))
    s.autotune(reps=1)
    V = _random(torch, 4, 12)
    Z, _ = s.apply_batch("SAP", 0, V, arg=1)
    Z = to_np(Z)
    for q in range(4):
        err = rel(Z[q].reshape(-1, 4, 3), o.sap(0, to_np(V[q]), 1))
        say("  96x48^3 FP32 SAP sweep, RHS %d of 4: %.2e" % (q, err))
        assert err < 1e-5


def test_c4_benchmark_solve_true_residual(c4):
    s, o, G, torch = c4
    s.setup(params=c4_params(G))
    s.autotune(reps=1)
    s.autotune_coarse(reps=1)
    vol = int(np.prod(DIMS))
    b = torch.zeros((4, vol, 4, 3), dtype=torch.complex128, device="cuda")
    for q in range(4):
        b[q, 0, q // 3, q % 3] = 1.0
    X, sts = s.solve_batch(b, 1e-10)
    X = to_np(X)
    bn = to_np(b)
    for q in range(4):
        r = bn[q] - o.apply(X[q])
        relres = float(np.linalg.norm(r) / np.linalg.norm(bn[q]))
        say("  point source %d: outer its %d, true residual (oracle D) %.3e, reported %.3e" %
            (q, sts[q]["outer_iters"], relres, sts[q]["true_relres"]))
        assert sts[q]["converged"] and relres <= 1e-10
        assert abs(relres - sts[q]["true_relres"]) <= 1e-3 * relres + 1e-14
