"""GPU parity at the full size of the 32^3 x 64 precision study: 64x32^3,
the device-drawn APE field, m0 = m_crit + 0.01 of this field, three levels
(aggregates 4^4 then 2^4, N = 20 / 20, SAP blocks 4^4 / 2^4, 4 MR steps),
with the oracle on the host on the same field.

* FP16 storage (operators and fine-level vectors in FP16 with per-site
  scales): one SAP sweep against the oracle's at the FP16 SAP bar of the
  small cases (1e-2 of the largest entry).
* Solves with the FP32 and with the FP16-storage preconditioner inside the
  FP64 outer FGMRES: true residual, with the oracle's D applied to the
  returned x, at most 1e-10; the FP16 form's solution within kappa * tol
  (reading A33: 1e-8) of the FP32 form's."""
import json
import os

import numpy as np
import pytest

from tests._gpu import rel, say, to_np

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DIMS = (64, 32, 32, 32)


def c3_params(G, precision):
    return G.default_params(levels=3, n_tv=[20, 20], agg=[(4, 4, 4, 4), (2, 2, 2, 2)],
                            sap=[(4, 4, 4, 4), (2, 2, 2, 2)], mr_steps=[4, 4], nu=2, n_inv=6, coarse_tol=5e-2,
                            coarse_restart=30, mid_tol=5e-2, mid_restart=10, outer_restart=25, precision=precision)


@pytest.fixture(scope="module")
def c3():
    import torch

    import oracle as O
    import paper_1303_1377_amd as G
    from paper_1303_1377_amd import fields as F

    with open(os.path.join(ROOT, "paper_1303_1377_amd", "mcrit_fields.json")) as f:
        m0 = json.load(f)["lat64x32c3_ape2_seed0_dev"]["m_crit"] + 0.01
    say("case: 64x32^3 full size, device field, m0 = %.6f" % m0)
    U = F.make_gauge_device(DIMS, 0.4, 0, ape_steps=2, ape_alpha=0.5)
    torch.cuda.synchronize()
    o = O.Oracle(DIMS, U.cpu().numpy(), m0, 1.0)
    o.configure(levels=2, n_tv=[1], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], mr_steps=[4])
    s = G.Solver(DIMS, U, m0, 1.0)
    del U
    yield s, o, G, torch
    s.close()
    o.close()
    torch.cuda.empty_cache()


def _gaussian(torch, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    vol = int(np.prod(DIMS))
    re = torch.randn((vol, 4, 3), generator=g, device="cuda", dtype=torch.float64)
    im = torch.randn((vol, 4, 3), generator=g, device="cuda", dtype=torch.float64)
    return torch.complex(re, im)


def test_c3_fp16_sap_sweep(c3):
    s, o, G, torch = c3
    s.configure(c3_params(G, 16))
    v = _gaussian(torch, 21)
    z, _ = s.apply("SAP", 0, v, arg=1)
    err = rel(to_np(z), o.sap(0, to_np(v), 1))
    say("  64x32^3 FP16-storage SAP sweep: %.2e" % err)
    assert 1e-5 < err < 1e-2


def test_c3_solves_fp32_and_fp16(c3):
    s, o, G, torch = c3
    b = _gaussian(torch, 22)
    bn = to_np(b)
    xs = {}
    for prec in (32, 16):
        s.setup(params=c3_params(G, prec))
        s.autotune(reps=1)
        x, st = s.solve(b, 1e-10)
        xn = to_np(x)
        relres = float(np.linalg.norm(bn - o.apply(xn)) / np.linalg.norm(bn))
        say("  precision %d: outer its %d, true residual (oracle D) %.3e, reported %.3e" %
            (prec, st["outer_iters"], relres, st["true_relres"]))
        assert st["converged"] and relres <= 1e-10
        xs[prec] = xn
    diff = float(np.linalg.norm(xs[16] - xs[32]) / np.linalg.norm(xs[32]))
    say("  |x_16 - x_32| / |x_32| = %.2e" % diff)
    assert diff <= 1e-8
