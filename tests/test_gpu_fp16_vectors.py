"""Precision 16 with FP16 spinor storage on the fine level: the V-cycle's
input, the interpolated and smoothed z and the outer FGMRES's preconditioned
vectors are stored in FP16 with one FP32 scale per site and chirality half
(the largest modulus of the half's 12 reals), arithmetic in FP32.

Bars.  A stored entry is off by at most half an FP16 ulp of the largest value
in [-1, 1], 2^-12 = 2.4e-4 of its half-site's largest modulus; the operators
are FP16 too (unit roundoff 2^-11 per entry, the 4e-3 bound of the FP16
operator test).  A V-cycle (restriction, 6 coarse GMRES iterations, prolongation,
two SAP sweeps) composes about ten such roundings, amplified by the fixed
coarse GMRES polynomial: bar 2e-2 of the largest entry, and above 1e-5 so that
the FP16 path is the one in use.  Solves: the FP64 outer FGMRES reaches 1e-10
and agrees with the oracle's solution within kappa * tol (reading A33, 1e-8).
Scale invariance: right-hand sides scaled by 1e-8 and 1e+12 (far outside the
FP16 range without the scales) converge in the same iteration count within
one."""
import numpy as np
import pytest

from paper_1303_1377_amd import fields as F
from tests._gpu import Pair, rel, say, to_np

pytestmark = pytest.mark.gpu

DIMS = (8, 8, 8, 8)
KW = dict(levels=2, n_tv=[8], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], mr_steps=[4], n_inv=3, outer_restart=20)


def test_fp16_vcycle_matches_oracle():
    say("case: precision-16 V-cycle (FP16 vectors) against the oracle, coarse fixed 6")
    p = Pair(DIMS, eps=0.3, seed=6, m0=-0.25, csw=1.0)
    p.configure(precision=16, levels=2, n_tv=[8], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], coarse_fixed=6)
    tv = p.vectors(0, 8, 7)
    p.o.set_vectors(0, tv)
    p.o.build(0)
    p.g.set_test_vectors(0, tv)
    p.g.build_level(0)
    p.o.mark_setup()
    p.g.mark_setup()
    for seed in (41, 42):
        r = F.gaussian_spinor(DIMS, seed)
        z, _ = p.g.apply("VCYCLE", 0, r)
        err = rel(to_np(z), p.o.vcycle(0, r))
        say("  seed %d: V-cycle error %.3e" % (seed, err))
        assert 1e-5 < err < 2e-2


def test_fp16_batch_solve_matches_oracle():
    say("case: precision-16 batch of 3 solves against the oracle's solutions")
    import paper_1303_1377_amd as G

    p = Pair(DIMS, eps=0.3, seed=3, m0=-0.25, csw=1.0)
    p.configure(precision=16, max_rhs=3, **KW)
    tv = p.vectors(0, 8, 5)
    p.g.set_test_vectors(0, tv)
    p.g.setup(params=G.default_params(precision=16, max_rhs=3, given_vectors=1, **KW))
    p.o.setup([tv])
    B = np.stack([F.gaussian_spinor(DIMS, 80 + i) for i in range(3)])
    X, sts = p.g.solve_batch(B, 1e-10)
    for i in range(3):
        x = to_np(X[i])
        relres = float(np.linalg.norm(B[i] - p.o.apply(x)) / np.linalg.norm(B[i]))
        xo, sto = p.o.solve(B[i], 1e-12)
        diff = float(np.linalg.norm(x - xo) / np.linalg.norm(xo))
        say("  rhs %d: its %d relres %.2e |x - x_o|/|x_o| %.2e" % (i, sts[i]["outer_iters"], relres, diff))
        assert sts[i]["converged"] and relres <= 1e-10 and diff <= 1e-8


def test_fp16_vectors_are_scale_invariant():
    say("case: precision-16 solves of b, 1e-8 b and 1e12 b")
    import paper_1303_1377_amd as G

    p = Pair(DIMS, eps=0.3, seed=3, m0=-0.25, csw=1.0)
    p.configure(precision=16, **KW)
    tv = p.vectors(0, 8, 5)
    p.g.set_test_vectors(0, tv)
    p.g.setup(params=G.default_params(precision=16, given_vectors=1, **KW))
    b = F.gaussian_spinor(DIMS, 90)
    its = {}
    for sc in (1.0, 1e-8, 1e12):
        x, st = p.g.solve(sc * b, 1e-10)
        x = to_np(x)
        relres = float(np.linalg.norm(sc * b - p.o.apply(x)) / np.linalg.norm(sc * b))
        its[sc] = st["outer_iters"]
        say("  scale %g: its %d relres %.2e" % (sc, st["outer_iters"], relres))
        assert st["converged"] and relres <= 1e-10
    assert abs(its[1e-8] - its[1.0]) <= 1 and abs(its[1e12] - its[1.0]) <= 1


def test_fp16_coarse_stencil_is_scale_invariant():
    """The matrix-core coarse stencil of precision 16 divides each right-hand
    side's inputs by their largest modulus over the site's 9-block stencil
    before rounding them to FP16: twelve vectors (nd = 40) scaled by 1e-9 and
    1e6, whose entries unscaled would fall below FP16's subnormals or above its
    range, give D_c and the Schur complement within the FP16-storage bound
    (4e-3) of the oracle's scaled result, as the unscaled vectors do."""
    say("case: precision-16 multi-RHS coarse stencil on vectors scaled by 1e-9 and 1e6")
    import paper_1303_1377_amd as G

    p = Pair(DIMS, eps=0.3, seed=8, m0=-0.25, csw=1.0)
    kw = dict(levels=2, n_tv=[20], agg=[(4, 4, 4, 4)], sap=[(4, 4, 4, 4)], mr_steps=[4], coarse_fixed=6)
    p.o.configure(**kw)
    p.g.configure(G.default_params(precision=16, max_rhs=12, **kw))
    tv = p.vectors(0, 20, 12)
    p.o.set_vectors(0, tv)
    p.o.build(0)
    p.g.set_test_vectors(0, tv)
    p.g.build_level(0)
    p.g.mark_setup()
    p.o.mark_setup()
    vol_c, ndc = p.o.level_size(1)
    rng = np.random.default_rng(31)
    V = rng.standard_normal((12, vol_c, ndc)) + 1j * rng.standard_normal((12, vol_c, ndc))
    refD = [p.o.apply(V[q], level=1) for q in range(12)]
    refS = [p.o.schur(1, V[q]) for q in range(12)]
    for f in (1.0, 1e-9, 1e6):
        D, _ = p.g.apply_batch("D", 1, f * V)
        S, _ = p.g.apply_batch("SCHUR", 1, f * V)
        D, S = to_np(D), to_np(S)
        ed = max(rel(D[q], f * refD[q]) for q in range(12))
        es = max(rel(S[q], f * refS[q]) for q in range(12))
        say("  scale %g: D_c error %.2e, Schur error %.2e" % (f, ed, es))
        assert ed < 4e-3 and es < 4e-3
