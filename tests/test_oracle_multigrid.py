"""Pins of the oracle's multigrid components: interpolation, coarse operator,
SAP, MR block solver, V-cycle and FGMRES, against the identities of the paper
(Lemma cgprops, the SAP and V-cycle error propagators) and dense linear algebra."""
import numpy as np
import pytest

import oracle as O
from paper_1303_1377_amd import fields as F
from tests import _dense as DN

DIMS = (4, 4, 2, 2)
VOL = 64
AGG = (2, 2, 2, 2)
SAPB = (2, 2, 2, 2)
NV = 4


def _make(m0=-0.25, csw=1.0, seed=3, **kw):
    U = F.make_gauge(DIMS, 0.35, seed)
    o = O.Oracle(DIMS, U, m0, csw)
    prm = dict(levels=2, n_tv=[NV], agg=[AGG], sap=[SAPB], mr_steps=[4])
    prm.update(kw)
    o.configure(**prm)
    return U, o


@pytest.fixture(scope="module")
def built():
    U, o = _make()
    tv = F.random_vectors(VOL, 12, NV, 21)
    o.set_vectors(0, tv)
    o.build(0)
    D = DN.dense_of(o.apply, VOL * 12)
    P = DN.dense_P(o.get_P(0), DIMS, AGG)
    (cd, ndc) = o.level_info(1)
    M, Mi = o.get_coarse(1)
    Dc = DN.dense_coarse(M, cd)
    return dict(U=U, o=o, tv=tv, D=D, P=P, Dc=Dc, M=M, Mi=Mi, cd=cd)


def test_P_orthonormal_and_range(built):
    """P^H P = I and each test vector lies in range(P) (Sec. 3.1)."""
    P = built["P"]
    assert np.abs(P.conj().T @ P - np.eye(P.shape[1])).max() < 1e-13
    for v in built["tv"]:
        v = v.reshape(-1)
        assert np.linalg.norm(P @ (P.conj().T @ v) - v) < 1e-12 * np.linalg.norm(v)


def test_P_gram_schmidt_order(built):
    """Local orthonormalisation in column order: Q^H W is upper triangular with
    positive diagonal for each aggregate (the unique such QR)."""
    o, tv = built["o"], built["tv"]
    Pc = o.get_P(0)
    ai, cd = DN.aggregate_index(DIMS, AGG)
    for a in range(int(np.prod(cd))):
        sites = np.where(ai == a)[0]
        for h in range(2):
            W = np.stack([tv[k][sites][:, 6 * h:6 * h + 6].reshape(-1) for k in range(NV)], axis=1)
            Q = np.stack([Pc[k][sites][:, 6 * h:6 * h + 6].reshape(-1) for k in range(NV)], axis=1)
            R = Q.conj().T @ W
            assert np.abs(np.tril(R, -1)).max() < 1e-12
            assert np.all(np.abs(np.diag(R).imag) < 1e-12) and np.all(np.diag(R).real > 0)


def test_gamma5_commutes_with_P(built):
    """eq. (commute_with_g5): Gamma5 P = P Gamma5^c for Gamma5-compatible aggregates."""
    P = built["P"]
    G5 = DN.gamma5_fine(VOL)
    G5c = DN.gamma5_coarse(P.shape[1] // (2 * NV), NV)
    assert np.abs(G5 @ P - P @ G5c).max() < 1e-14


def test_Dc_is_galerkin_product(built):
    """The assembled stencil equals the explicit product P^H D P."""
    D, P, Dc = built["D"], built["P"], built["Dc"]
    ref = P.conj().T @ D @ P
    assert np.abs(Dc - ref).max() < 1e-13 * np.abs(ref).max()


def test_Dc_gamma5c_symmetric(built):
    """Lemma cgprops (iii): Gamma5^c D_c is Hermitian."""
    Dc = built["Dc"]
    G5c = DN.gamma5_coarse(Dc.shape[0] // (2 * NV), NV)
    H = G5c @ Dc
    assert np.abs(H - H.conj().T).max() < 1e-13


def test_field_of_values_inclusion(built):
    """Lemma cgprops (iv): F(D_c) subset F(D): for every direction theta the
    support function max Re(e^{i theta} z) over F(D_c) is at most that of F(D)."""
    D, Dc = built["D"], built["Dc"]
    for th in np.linspace(0, 2 * np.pi, 13):
        h = lambda A: np.linalg.eigvalsh(0.5 * (np.exp(1j * th) * A + (np.exp(1j * th) * A).conj().T)).max()
        assert h(Dc) <= h(D) + 1e-12


def test_petrov_galerkin_equals_galerkin(built):
    """Lemma cgprops (i),(ii): with R = (Gamma5 P)^H, D_c^PG = Gamma5^c D_c and the
    two coarse-grid corrections coincide."""
    D, P, Dc = built["D"], built["P"], built["Dc"]
    G5 = DN.gamma5_fine(VOL)
    G5c = DN.gamma5_coarse(Dc.shape[0] // (2 * NV), NV)
    R = (G5 @ P).conj().T
    Dpg = R @ D @ P
    assert np.abs(Dpg - G5c @ Dc).max() < 1e-13
    n = D.shape[0]
    E1 = np.eye(n) - P @ np.linalg.solve(Dc, P.conj().T @ D)
    E2 = np.eye(n) - P @ np.linalg.solve(Dpg, R @ D)
    assert np.abs(E1 - E2).max() < 1e-10
    # the coarse-grid correction is a projection (Sec. 3)
    assert np.abs(E1 @ E1 - E1).max() < 1e-10


def test_Dc_mass_shift(built):
    """P^H P = I implies D_c(m0 + d) = D_c(m0) + d I."""
    U, o, tv = built["U"], built["o"], built["tv"]
    _, o2 = _make(m0=-0.25 + 0.2)
    o2.set_vectors(0, tv)
    o2.build(0)
    M2, _ = o2.get_coarse(1)
    Dc2 = DN.dense_coarse(M2, built["cd"])
    assert np.abs(Dc2 - built["Dc"] - 0.2 * np.eye(Dc2.shape[0])).max() < 1e-13


def test_restrict_prolong(built):
    o, P = built["o"], built["P"]
    rng = np.random.default_rng(0)
    v = rng.standard_normal(VOL * 12) + 1j * rng.standard_normal(VOL * 12)
    assert np.abs(o.restrict(0, v).reshape(-1) - P.conj().T @ v).max() < 1e-13
    vc = rng.standard_normal(P.shape[1]) + 1j * rng.standard_normal(P.shape[1])
    assert np.abs(o.prolong(0, vc).reshape(-1) - P @ vc).max() < 1e-13


def test_coarse_self_inverse(built):
    M, Mi = built["M"], built["Mi"]
    for c in range(M.shape[0]):
        assert np.abs(M[c, 0] @ Mi[c] - np.eye(M.shape[2])).max() < 1e-12


def _block_dense(D, sites):
    idx = np.concatenate([np.arange(12 * s, 12 * s + 12) for s in sites])
    return idx, D[np.ix_(idx, idx)]


def test_block_solve_exact_limit_and_even_residual():
    """MR block solver (Sec. 5): the block residual vanishes on the block's even
    sites for any number of steps; it is non-increasing in the number of steps;
    many steps give the exact block solution D_i^{-1} r_i (eq. localsystem)."""
    U, o = _make(m0=0.3)
    D = DN.dense_of(o.apply, VOL * 12)
    bid, _ = DN.block_masks(DIMS, SAPB)
    x = DN.coords(DIMS)
    par = x.sum(axis=1) % 2
    rng = np.random.default_rng(7)
    r = rng.standard_normal(VOL * 12) + 1j * rng.standard_normal(VOL * 12)
    blk = 2
    sites = np.where(bid == blk)[0]
    idx, Di = _block_dense(D, sites)
    prev = np.inf
    for steps in (1, 2, 3, 4, 6, 8):
        o.configure(levels=2, n_tv=[NV], agg=[AGG], sap=[SAPB], mr_steps=[steps])
        z = o.block_solve(0, blk, r).reshape(-1)
        e = z[idx]
        res = r[idx] - Di @ e
        ev = np.concatenate([np.arange(12 * i, 12 * i + 12) for i, s in enumerate(sites) if par[s] == 0])
        assert np.abs(res[ev]).max() < 1e-13 * np.abs(r).max()
        n = np.linalg.norm(res)
        assert n <= prev * (1 + 1e-12)
        prev = n
        outside = np.setdiff1d(np.arange(VOL * 12), idx)
        assert np.abs(z[outside]).max() == 0.0
    o.configure(levels=2, n_tv=[NV], agg=[AGG], sap=[SAPB], mr_steps=[300])
    z = o.block_solve(0, blk, r).reshape(-1)
    exact = np.linalg.solve(Di, r[idx])
    assert np.linalg.norm(z[idx] - exact) < 1e-10 * np.linalg.norm(exact)


def _sap_dense(D, bid, col):
    n = D.shape[0]
    B = [np.zeros((n, n), dtype=np.complex128) for _ in range(2)]
    for b in np.unique(bid):
        sites = np.where(bid == b)[0]
        idx, Di = _block_dense(D, sites)
        c = col[sites[0]]
        B[c][np.ix_(idx, idx)] += np.linalg.inv(Di)
    return B


def test_sap_error_propagator():
    """Sec. 2.3: with exact block solves one SAP iteration is
    z <- (I - K D) z + K b with K = B_black (I - D B_red) + B_red, and
    M_SAP^(nu) = sum_{k<nu} (I - K D)^k K."""
    U, o = _make(m0=0.3, mr_steps=[300])
    D = DN.dense_of(o.apply, VOL * 12)
    bid, col = DN.block_masks(DIMS, SAPB)
    Bred, Bblack = _sap_dense(D, bid, col)
    n = D.shape[0]
    K = Bblack @ (np.eye(n) - D @ Bred) + Bred
    E = np.eye(n) - K @ D
    # E_SAP = (I - B_black D)(I - B_red D)
    assert np.abs(E - (np.eye(n) - Bblack @ D) @ (np.eye(n) - Bred @ D)).max() < 1e-10
    rng = np.random.default_rng(1)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for nu in (1, 2, 3):
        Mnu = sum(np.linalg.matrix_power(E, k) for k in range(nu)) @ K
        z = o.sap(0, b, nu).reshape(-1)
        assert np.linalg.norm(z - Mnu @ b) < 1e-9 * np.linalg.norm(Mnu @ b)
    # from a nonzero start: z1 = E z0 + K b
    z0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    z = o.sap(0, b, 1, z0=z0).reshape(-1)
    assert np.linalg.norm(z - (E @ z0 + K @ b)) < 1e-9 * np.linalg.norm(z)


def test_sap_single_block_is_inverse():
    """A single SAP block spanning the lattice: M_SAP = D^{-1}."""
    U, o = _make(m0=0.4, sap=[DIMS], mr_steps=[2000])
    D = DN.dense_of(o.apply, VOL * 12)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(VOL * 12) + 1j * rng.standard_normal(VOL * 12)
    z = o.sap(0, b, 1).reshape(-1)
    x = np.linalg.solve(D, b)
    assert np.linalg.norm(z - x) < 1e-8 * np.linalg.norm(x)


def test_vcycle_linearised_equals_formula():
    """eq. (iterationmatrix): with exact block and coarse solves the V-cycle is
    C = M_SAP^(nu) + P D_c^{-1} P^H - M_SAP^(nu) D P D_c^{-1} P^H = M pi_L + P D_c^{-1} P^H."""
    U, o = _make(m0=0.3, mr_steps=[300], coarse_tol=1e-14, coarse_restart=64, coarse_maxit=5000)
    tv = F.random_vectors(VOL, 12, NV, 5)
    o.set_vectors(0, tv)
    o.build(0)
    D = DN.dense_of(o.apply, VOL * 12)
    P = DN.dense_P(o.get_P(0), DIMS, AGG)
    cd, _ = o.level_info(1)
    Dc = DN.dense_coarse(o.get_coarse(1)[0], cd)
    bid, col = DN.block_masks(DIMS, SAPB)
    Bred, Bblack = _sap_dense(D, bid, col)
    n = D.shape[0]
    K = Bblack @ (np.eye(n) - D @ Bred) + Bred
    E = np.eye(n) - K @ D
    M2 = (np.eye(n) + E) @ K
    CGC = P @ np.linalg.solve(Dc, P.conj().T)
    C = M2 + CGC - M2 @ D @ CGC
    piL = np.eye(n) - D @ CGC
    assert np.abs(C - (M2 @ piL + CGC)).max() < 1e-9
    rng = np.random.default_rng(4)
    r = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    z = o.vcycle(0, r).reshape(-1)
    assert np.linalg.norm(z - C @ r) < 1e-9 * np.linalg.norm(C @ r)


def test_coarse_solver_residual_and_oe_exact():
    """Odd-even GMRES on D_c: the requested relative residual is reached, and a
    tiny tolerance reproduces the dense solution."""
    U, o = _make(m0=-0.1)
    o.set_vectors(0, F.random_vectors(VOL, 12, NV, 8))
    o.build(0)
    cd, ndc = o.level_info(1)
    Dc = DN.dense_coarse(o.get_coarse(1)[0], cd)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(Dc.shape[0]) + 1j * rng.standard_normal(Dc.shape[0])
    e, its = o.coarse_solve(1, r)
    assert its >= 1
    # residual of the odd-even reduced system: even part exactly zero after the
    # back-substitution, odd part reduced by the factor 20 relative to f_o
    xc = DN.coords(cd)
    par = np.repeat(xc.sum(axis=1) % 2, ndc)
    ev, od = np.where(par == 0)[0], np.where(par == 1)[0]
    f_o = r[od] - Dc[np.ix_(od, ev)] @ np.linalg.solve(Dc[np.ix_(ev, ev)], r[ev])
    res = r - Dc @ e
    assert np.abs(res[ev]).max() < 1e-12 * np.abs(r).max()
    assert np.linalg.norm(res[od]) <= 5e-2 * np.linalg.norm(f_o) * (1 + 1e-10)
    o.configure(levels=2, n_tv=[NV], agg=[AGG], sap=[SAPB], mr_steps=[4], coarse_tol=1e-14, coarse_maxit=10000)
    o.set_vectors(0, F.random_vectors(VOL, 12, NV, 8))
    o.build(0)
    e, its = o.coarse_solve(1, r)
    ex = np.linalg.solve(Dc, r)
    assert np.linalg.norm(e - ex) < 1e-11 * np.linalg.norm(ex)


def test_schur_complement_dense():
    """Odd-even Schur complement S = A_oo - D_oe A_ee^{-1} D_eo of D_c."""
    U, o = _make()
    o.set_vectors(0, F.random_vectors(VOL, 12, NV, 8))
    o.build(0)
    cd, ndc = o.level_info(1)
    Dc = DN.dense_coarse(o.get_coarse(1)[0], cd)
    xc = DN.coords(cd)
    par = np.repeat(xc.sum(axis=1) % 2, ndc)
    e, od = np.where(par == 0)[0], np.where(par == 1)[0]
    S = Dc[np.ix_(od, od)] - Dc[np.ix_(od, e)] @ np.linalg.solve(Dc[np.ix_(e, e)], Dc[np.ix_(e, od)])
    rng = np.random.default_rng(9)
    v = np.zeros(Dc.shape[0], dtype=np.complex128)
    v[od] = rng.standard_normal(len(od)) + 1j * rng.standard_normal(len(od))
    out = o.schur(1, v)
    assert np.abs(out[od] - S @ v[od]).max() < 1e-12
    assert np.abs(out[e]).max() == 0.0


def test_dense_direct_solve_2x4():
    """Full DD-alpha-AMG solve on a 2^4 lattice equals the dense direct solution
    (single 2^4 aggregate and SAP block)."""
    dims = (2, 2, 2, 2)
    U = F.make_gauge(dims, 0.3, 0)
    o = O.Oracle(dims, U, -0.2, 1.0)
    o.configure(levels=2, n_tv=[4], agg=[(2, 2, 2, 2)], sap=[(2, 2, 2, 2)], mr_steps=[4], n_inv=2, outer_restart=20)
    o.setup([F.random_vectors(16, 12, 4, 1)])
    b = F.gaussian_spinor(dims, 1000)
    x, st = o.solve(b, 1e-10)
    D = DN.dense_of(o.apply, 192)
    ex = np.linalg.solve(D, b.reshape(-1))
    assert st["converged"] and st["true_relres"] <= 1e-10
    kappa = np.linalg.cond(D)
    assert np.linalg.norm(x.reshape(-1) - ex) <= 2 * kappa * 1e-10 * np.linalg.norm(ex)


@pytest.mark.slow
def test_solve_4x4_matches_dense_and_setup_invariants():
    """Configuration-1 sizes: 4^4, 2 levels, aggregates and SAP blocks 2^4, N=8,
    m0=-0.4, csw=1, FGMRES(20) to 1e-10.  The solution agrees with dense LU
    within kappa*tol; setup output keeps P^H P = I and range(P) contains the
    final test vectors."""
    dims = (4, 4, 4, 4)
    U = F.make_gauge(dims, 0.3, 0)
    o = O.Oracle(dims, U, -0.4, 1.0)
    o.configure(levels=2, n_tv=[8], agg=[(2, 2, 2, 2)], sap=[(2, 2, 2, 2)], mr_steps=[4], n_inv=6,
                outer_restart=20)
    o.setup([F.random_vectors(256, 12, 8, 2024)])
    b = F.gaussian_spinor(dims, 1000)
    x, st = o.solve(b, 1e-10)
    assert st["converged"] and st["true_relres"] <= 1e-10
    D = DN.dense_of(o.apply, 3072)
    ex = np.linalg.solve(D, b.reshape(-1))
    kappa = np.linalg.cond(D)
    assert np.linalg.norm(x.reshape(-1) - ex) <= 2 * kappa * 1e-10 * np.linalg.norm(ex)
    P = DN.dense_P(o.get_P(0), dims, (2, 2, 2, 2))
    assert np.abs(P.conj().T @ P - np.eye(P.shape[1])).max() < 1e-12
    for v in o.get_vectors(0):
        v = v.reshape(-1)
        assert abs(np.linalg.norm(v) - 1) < 1e-12
        assert np.linalg.norm(P @ (P.conj().T @ v) - v) < 1e-10


def test_coarse_level_sap_error_propagator():
    """SAP on the coarse operator (intermediate level of a 3-level hierarchy):
    with exact block solves it follows the same error propagator as on the
    fine level, with the dense site blocks of D_c."""
    dims = (8, 4, 4, 4)
    U = F.make_gauge(dims, 0.35, 4)
    o = O.Oracle(dims, U, 0.3, 1.0)
    o.configure(levels=3, n_tv=[4, 4], agg=[(2, 2, 2, 2), (2, 2, 2, 2)], sap=[(2, 2, 2, 2), (2, 2, 2, 2)],
                mr_steps=[4, 400])
    o.set_vectors(0, F.random_vectors(512, 12, 4, 6))
    o.build(0)
    cd, ndc = o.level_info(1)
    assert cd == (4, 2, 2, 2) and ndc == 8
    Dc = DN.dense_coarse(o.get_coarse(1)[0], cd)
    xc = DN.coords(cd)
    bc = xc // 2
    nbk = [cd[m] // 2 for m in range(4)]
    bid = DN.site_index(nbk, bc)
    col = bc.sum(axis=1) % 2
    n = Dc.shape[0]
    B = [np.zeros((n, n), dtype=np.complex128) for _ in range(2)]
    for b in np.unique(bid):
        sites = np.where(bid == b)[0]
        idx = np.concatenate([np.arange(ndc * s, ndc * s + ndc) for s in sites])
        B[col[sites[0]]][np.ix_(idx, idx)] += np.linalg.inv(Dc[np.ix_(idx, idx)])
    K = B[1] @ (np.eye(n) - Dc @ B[0]) + B[0]
    E = np.eye(n) - K @ Dc
    rng = np.random.default_rng(2)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    z = o.sap(1, b, 2).reshape(-1)
    ref = (np.eye(n) + E) @ K @ b
    assert np.linalg.norm(z - ref) < 1e-9 * np.linalg.norm(ref)


@pytest.mark.slow
def test_three_level_solve_converges():
    """Three levels (recursive two-level method on D_c): the outer FGMRES
    reaches the requested true residual."""
    dims = (8, 8, 4, 4)
    U = F.make_gauge(dims, 0.3, 7)
    o = O.Oracle(dims, U, -0.2, 1.0)
    o.configure(levels=3, n_tv=[6, 6], agg=[(2, 2, 2, 2), (2, 2, 2, 2)], sap=[(2, 2, 2, 2), (2, 2, 2, 2)],
                mr_steps=[4, 4], n_inv=3, outer_restart=20)
    vol = 1024
    o.setup([F.random_vectors(vol, 12, 6, 1), F.random_vectors(vol // 16, 12, 6, 2)])
    b = F.gaussian_spinor(dims, 1000)
    x, st = o.solve(b, 1e-10)
    assert st["converged"] and st["true_relres"] <= 1e-10
    assert st["coarse_iters"][1] > 0 and st["coarse_iters"][2] > 0
