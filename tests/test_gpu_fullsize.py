"""GPU parity at the full size of the benchmarked workload: the 16^4 lattice
with its APE-smeared field and mass (m_crit + 0.02), the benchmark's
parameters (two levels, aggregates and SAP blocks 4^4, N = 20, 3 MR steps,
FP64) and the launch schedule the benchmark's autotuner picks.  At this size
the FP64 oracle still computes every output in seconds, so the comparisons
are element by element over the whole lattice, at the bars of the small
cases: linear operator applies 1e-13 (FP64) / 2e-6 (FP32), SAP 1e-12 (FP32: 1e-5), coarse
GMRES with a fixed iteration count 1e-10; the full solve is checked by its
true residual under the oracle's operator (<= 1e-10) and its solution against
the oracle's own solution (its own setup, tolerance 1e-12): two solutions that
meet the true residual agree to about kappa * tol (reading A33: <= 1e-8)."""
import json
import os

import numpy as np
import pytest

from paper_1303_1377_amd import fields as F
from tests._gpu import rel, say, to_np

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PARAMS = dict(levels=2, n_tv=[20], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], mr_steps=[3], nu=2, n_inv=6,
              coarse_tol=5e-2, coarse_restart=30, outer_restart=25)


class Full:
    def __init__(self):
        import oracle as O
        import paper_1303_1377_amd as G

        with open(os.path.join(ROOT, "tests", "golden", "mcrit.json")) as f:
            info = json.load(f)["lat16x4_ape2_seed0"]
        self.dims = tuple(info["dims"])
        self.m0 = info["m_crit"] + 0.02
        self.csw = info["csw"]
        self.U = F.make_gauge(self.dims, info["eps"], info["seed"], ape_steps=info["ape"], ape_alpha=0.5)
        self.o = O.Oracle(self.dims, self.U, self.m0, self.csw)
        self.g = G.Solver(self.dims, self.U, self.m0, self.csw)
        self.G = G

    def configure(self, precision=64, **over):
        kw = dict(PARAMS)
        kw.update(over)
        self.o.configure(**{k: v for k, v in kw.items() if k != "precision"})
        self.g.configure(self.G.default_params(precision=precision, **kw))
        sched, _ = self.g.autotune(reps=1)
        say("full size: schedule", sched)

    def inject(self, seed=7):
        vol, nd = self.o.level_size(0)
        tv = F.random_vectors(vol, nd, 20, seed)
        self.o.set_vectors(0, tv)
        self.o.build(0)
        self.g.set_test_vectors(0, tv)
        self.g.build_level(0)


@pytest.fixture(scope="module")
def full():
    say("case: full size 16^4, the benchmarked field and parameters")
    return Full()


def test_fullsize_stencil(full):
    full.configure()
    b = F.gaussian_spinor(full.dims, 31)
    ref = full.o.apply(b)
    y, _ = full.g.apply("D", 0, b)
    assert rel(to_np(y), ref) < 1e-13
    full.configure(precision=32)
    y32, _ = full.g.apply("D_PREC", 0, b)
    assert rel(to_np(y32), ref) < 2e-6


def test_fullsize_sap(full):
    full.configure()
    b = F.gaussian_spinor(full.dims, 32)
    z, _ = full.g.apply("SAP", 0, b, arg=2)
    assert rel(to_np(z), full.o.sap(0, b, 2)) < 1e-12


def test_fullsize_sap_fp32(full):
    """The FP32 SAP kernel (two waves per SIMD, 4^4 blocks) at full size, at
    the FP32 SAP bar of the small cases."""
    full.configure(precision=32)
    b = F.gaussian_spinor(full.dims, 36)
    z, _ = full.g.apply("SAP", 0, b, arg=2)
    assert rel(to_np(z), full.o.sap(0, b, 2)) < 1e-5


def test_fullsize_transfer_and_coarse(full):
    full.configure(coarse_fixed=30)
    full.inject()
    assert rel(to_np(full.g.get_P(0)), full.o.get_P(0)) < 1e-12
    M, Mi = full.g.get_coarse(1)
    Mo, Mio = full.o.get_coarse(1)
    assert rel(to_np(M), Mo) < 1e-12
    assert rel(to_np(Mi), Mio) < 1e-10
    v = F.gaussian_spinor(full.dims, 33)
    rc, _ = full.g.apply("RESTRICT", 0, v)
    assert rel(to_np(rc), full.o.restrict(0, v)) < 1e-13
    vol_c, ndc = full.o.level_size(1)
    rng = np.random.default_rng(34)
    vc = rng.standard_normal((vol_c, ndc)) + 1j * rng.standard_normal((vol_c, ndc))
    pr, _ = full.g.apply("PROLONG", 0, vc)
    assert rel(to_np(pr), full.o.prolong(0, vc)) < 1e-13
    dc, _ = full.g.apply("D", 1, vc)
    assert rel(to_np(dc), full.o.apply(vc, level=1)) < 1e-13
    sc, _ = full.g.apply("SCHUR", 1, vc)
    assert rel(to_np(sc), full.o.schur(1, vc)) < 1e-13
    e, its = full.g.apply("COARSE_SOLVE", 1, vc)
    eo, itso = full.o.coarse_solve(1, vc)
    assert its == itso == 30
    assert rel(to_np(e), eo) < 1e-10


def test_fullsize_solve_true_residual(full):
    full.configure()
    full.g.setup(params=full.G.default_params(precision=64, **PARAMS))
    full.g.autotune(reps=1)
    full.g.autotune_coarse(reps=1)
    b = F.gaussian_spinor(full.dims, 35)
    x, st = full.g.solve(b, 1e-10)
    say("full size solve:", st["outer_iters"], st["true_relres"])
    assert st["converged"]
    r = b - full.o.apply(to_np(x))
    relres = float(np.linalg.norm(r) / np.linalg.norm(b))
    assert relres <= 1e-10
    assert abs(relres - st["true_relres"]) <= 1e-3 * relres + 1e-14


def test_fullsize_solution_matches_oracle_solution(full):
    """x of the benchmarked solve against the oracle's x for the same b."""
    full.configure()
    full.g.setup(params=full.G.default_params(precision=64, **PARAMS))
    b = F.gaussian_spinor(full.dims, 35)
    x, st = full.g.solve(b, 1e-10)
    okw = dict(PARAMS, n_inv=2)
    full.o.configure(**okw)
    full.o.setup([F.random_vectors(int(np.prod(full.dims)), 12, 20, 123)])
    xo, sto = full.o.solve(b, 1e-12)
    assert sto["converged"]
    diff = float(np.linalg.norm(to_np(x) - xo) / np.linalg.norm(xo))
    say("full size: |x - x_oracle| / |x_oracle| = %.3e (gpu its %d, oracle its %d)" %
        (diff, st["outer_iters"], sto["outer_iters"]))
    assert st["converged"] and diff <= 1e-8
