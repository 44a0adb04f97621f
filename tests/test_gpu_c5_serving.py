"""The serving workload at its real field sizes: one field of each C5 lattice
(16^4 two levels; 48x24^3 three levels with SAP blocks 2x3^3 on level 1 and a
coarsest 6x3^3 lattice; 64x32^3 three levels), each at m_crit + shift of its
own field, FP32 preconditioner, 4 continuous-batching slots per field, under a
200 GB budget.  Requests of 1-4 Gaussian right-hand sides arrive while others
run; every returned solution is checked with the oracle's D on the host (true
residual at most 1e-10, equal to the reported one) and the server's latency
statistics cover every request."""
import numpy as np
import pytest

from tests._gpu import say

pytestmark = pytest.mark.gpu


def test_serving_three_field_sizes_with_oracle_residuals():
    import torch

    import oracle as O
    import paper_1303_1377_amd as G
    from paper_1303_1377_amd import fields as F
    from paper_1303_1377_amd.serve_bench import field_params, field_table
    from paper_1303_1377_amd.serving import Server

    table = field_table(False)
    chosen = [table[0], table[2], table[4]]     # 16^4 seed 0, 48x24^3 seed 2, 64x32^3 seed 4
    say("case: serving at C5 sizes:", [(f["dims"], f["seed"], round(f["m0"], 6), f["levels"]) for f in chosen])
    U = {}
    for i, f in enumerate(chosen):
        U[i] = (F.make_gauge_device(f["dims"], 0.4, f["seed"], ape_steps=2, ape_alpha=0.5) if f["device"] else
                F.make_gauge(f["dims"], 0.4, f["seed"], ape_steps=2, ape_alpha=0.5))
    srv = Server(budget_bytes=200e9, max_rhs=4)
    for i, f in enumerate(chosen):
        srv.add_field(i, f["dims"], U[i], f["m0"], 1.0, params=field_params(G, f, 32, 4))

    def rhs(f, k, seed):
        d = f["dims"]
        g = torch.Generator(device="cuda").manual_seed(seed)
        vol = d[0] * d[1] * d[2] * d[3]
        re = torch.randn((k, vol, 4, 3), dtype=torch.float64, device="cuda", generator=g)
        im = torch.randn((k, vol, 4, 3), dtype=torch.float64, device="cuda", generator=g)
        return torch.complex(re, im)

    rng = np.random.default_rng(7)
    reqs = []
    for r in range(9):
        fi = r % 3
        k = int(rng.integers(1, 5))
        b = rhs(chosen[fi], k, 500 + r)
        reqs.append((fi, b, srv.submit(fi, b)))
    out = [(fi, b, fu.result(timeout=600)) for fi, b, fu in reqs]
    st = srv.stats()
    srv.close()
    say("  serving stats:", {k: st[k] for k in ("requests", "p50_latency_s", "p99_latency_s") if k in st})
    assert st["requests"] == 9 and st["p99_latency_s"] >= st["p50_latency_s"] > 0
    for fi, f in enumerate(chosen):
        Uh = U[fi].cpu().numpy() if hasattr(U[fi], "cpu") else U[fi]
        orc = O.Oracle(f["dims"], Uh, f["m0"], 1.0)
        worst = 0.0
        for gi, b, (x, sts) in out:
            if gi != fi:
                continue
            bn, xn = b.cpu().numpy(), x.cpu().numpy()
            for q in range(len(bn)):
                relres = float(np.linalg.norm(bn[q] - orc.apply(xn[q])) / np.linalg.norm(bn[q]))
                worst = max(worst, relres)
                assert sts[q]["converged"] and relres <= 1e-10
                assert abs(relres - sts[q]["true_relres"]) <= 1e-3 * relres + 1e-14
        orc.close()
        say("  field %s: largest true residual (oracle D) %.3e" % ("x".join(map(str, f["dims"])), worst))
