"""Coarse lattices with an odd extent (the third level of a 48 x 24^3 lattice
is 6 x 3^3): the coarsest level then has no odd-even structure and runs plain
GMRES on D_c (lexicographic layout), and an intermediate level whose extents
admit no power-of-two SAP blocks with two colours uses 2 x 3^3 SAP blocks
from site tables.  Against the oracle, which takes the same readings (plain
GMRES when a coarse extent is odd; SAP blocks of any extent with two colours):
operators to 1e-12, the coarse SAP to 1e-12, fixed-count coarse GMRES and
V-cycles to 1e-10 / 1e-9, and full solves to the 1e-10 true residual."""
import numpy as np
import pytest

from paper_1303_1377_amd import fields as F
from tests._gpu import Pair, rel, say, to_np

pytestmark = pytest.mark.gpu

DIMS = (8, 12, 12, 12)


def _inject(p, levels):
    for l in range(levels - 1):
        tv = p.vectors(l, p.o.params.n_tv[l], 40 + l)
        p.o.set_vectors(l, tv)
        p.o.build(l)
        p.g.set_test_vectors(l, tv)
        p.g.build_level(l)
    p.g.mark_setup()
    p.o.mark_setup()


def test_two_levels_odd_coarsest():
    """8 x 12^3 with 4^4 aggregates: coarsest lattice 2 x 3^3 (plain GMRES)."""
    say("case: two levels, coarsest 2x3^3")
    p = Pair(DIMS, eps=0.3, seed=3, m0=-0.15, csw=1.0)
    kw = dict(levels=2, n_tv=[6], agg=[(4, 4, 4, 4)], sap=[(2, 2, 2, 2)], mr_steps=[4], coarse_fixed=12)
    p.configure(**kw)
    assert p.g.level_info(1) == ((2, 3, 3, 3), 12)
    _inject(p, 2)
    M, Mi = p.g.get_coarse(1)
    Mo, Mio = p.o.get_coarse(1)
    assert rel(to_np(M), Mo) < 1e-12 and rel(to_np(Mi), Mio) < 1e-10
    vol1, nd1 = p.o.level_size(1)
    rng = np.random.default_rng(1)
    v = rng.standard_normal((vol1, nd1)) + 1j * rng.standard_normal((vol1, nd1))
    dc, _ = p.g.apply("D", 1, v)
    assert rel(to_np(dc), p.o.apply(v, level=1)) < 1e-13
    e, its = p.g.apply("COARSE_SOLVE", 1, v)
    eo, itso = p.o.coarse_solve(1, v)
    say("  coarse GMRES its", its, itso, "err", rel(to_np(e), eo))
    assert its == itso == 12 and rel(to_np(e), eo) < 1e-10
    r = F.gaussian_spinor(DIMS, 5)
    z, _ = p.g.apply("VCYCLE", 0, r)
    assert rel(to_np(z), p.o.vcycle(0, r)) < 1e-9


def test_three_levels_table_sap_and_odd_coarsest():
    """8 x 12^3 -> 4 x 6^3 (SAP blocks 2 x 3^3) -> 2 x 3^3 (plain GMRES)."""
    say("case: three levels, 2x3^3 SAP blocks on 4x6^3, coarsest 2x3^3")
    p = Pair(DIMS, eps=0.3, seed=4, m0=-0.15, csw=1.0)
    kw = dict(levels=3, n_tv=[6, 6], agg=[(2, 2, 2, 2), (2, 2, 2, 2)], sap=[(2, 2, 2, 2), (2, 3, 3, 3)],
              mr_steps=[4, 4], coarse_fixed=10, mid_fixed=3)
    p.configure(**kw)
    assert p.g.level_info(1) == ((4, 6, 6, 6), 12) and p.g.level_info(2) == ((2, 3, 3, 3), 12)
    _inject(p, 3)
    assert rel(to_np(p.g.get_coarse(2)[0]), p.o.get_coarse(2)[0]) < 1e-12
    vol1, nd1 = p.o.level_size(1)
    rng = np.random.default_rng(2)
    v1 = rng.standard_normal((vol1, nd1)) + 1j * rng.standard_normal((vol1, nd1))
    z1, _ = p.g.apply("SAP", 1, v1, arg=2)
    err = rel(to_np(z1), p.o.sap(1, v1, 2))
    say("  level-1 SAP (2x3^3 blocks) error %.3e" % err)
    assert err < 1e-12
    e, its = p.g.apply("FGMRES", 1, v1)
    eo, itso = p.o.fgmres_level(1, v1)
    assert its == itso == 3 and rel(to_np(e), eo) < 1e-10
    r = F.gaussian_spinor(DIMS, 6)
    z, _ = p.g.apply("VCYCLE", 0, r)
    assert rel(to_np(z), p.o.vcycle(0, r)) < 1e-9


@pytest.mark.parametrize("precision,bar", [(64, 1e-12), (32, 1e-5)])
def test_table_sap_two_rows_per_thread(precision, bar):
    """N = 20 on the fine level: 2 x 3^3 blocks of 40-dof sites need 1080 rows,
    more than a workgroup, so each thread carries two rows."""
    say("case: 2x3^3 coarse SAP with 40 unknowns per site, precision", precision)
    p = Pair(DIMS, eps=0.3, seed=6, m0=-0.15, csw=1.0)
    kw = dict(levels=3, n_tv=[20, 4], agg=[(2, 2, 2, 2), (2, 2, 2, 2)], sap=[(2, 2, 2, 2), (2, 3, 3, 3)],
              mr_steps=[4, 4])
    p.configure(precision=precision, **kw)
    assert p.g.level_info(1) == ((4, 6, 6, 6), 40)
    _inject(p, 3)
    vol1, nd1 = p.o.level_size(1)
    rng = np.random.default_rng(3)
    v1 = rng.standard_normal((vol1, nd1)) + 1j * rng.standard_normal((vol1, nd1))
    z1, _ = p.g.apply("SAP", 1, v1, arg=2)
    err = rel(to_np(z1), p.o.sap(1, v1, 2))
    say("  error %.3e" % err)
    assert err < bar


@pytest.mark.parametrize("precision", [64, 32])
def test_three_level_solve_with_odd_coarsest(precision):
    import paper_1303_1377_amd as G

    say("case: three-level solve 8x12^3, precision", precision)
    p = Pair(DIMS, eps=0.3, seed=4, m0=-0.15, csw=1.0)
    p.g.setup(params=G.default_params(precision=precision, levels=3, n_tv=[8, 8], agg=[(2, 2, 2, 2), (2, 2, 2, 2)],
                                      sap=[(2, 2, 2, 2), (2, 3, 3, 3)], mr_steps=[4, 4], n_inv=3, outer_restart=20,
                                      max_rhs=2))
    b = F.gaussian_spinor(DIMS, 7)
    x, st = p.g.solve(b, 1e-10)
    r = b - p.o.apply(to_np(x))
    relres = float(np.linalg.norm(r) / np.linalg.norm(b))
    say("  its", st["outer_iters"], "coarse", st["coarse_iters"][:3], "relres %.2e" % relres)
    assert st["converged"] and relres <= 1e-10
    B = np.stack([F.gaussian_spinor(DIMS, 8), F.gaussian_spinor(DIMS, 9)])
    X, sts = p.g.solve_batch(B, 1e-10)
    for q in range(2):
        rq = B[q] - p.o.apply(to_np(X[q]))
        assert sts[q]["converged"] and np.linalg.norm(rq) <= 1e-10 * np.linalg.norm(B[q])
