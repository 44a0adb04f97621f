"""Pins of the oracle's second comparison solver, inexact deflation (Sec. 4.1).

* The deflated operator: D pi_R with pi_R = I - P D_c^{-1} P^H D, against the
  same product formed from dense matrices (D column by column, P from its
  aggregate columns, D_c^{-1} by a dense inverse), with the coarse systems of
  the oracle solved to 1e-13 (4^4, aggregates 2^4).
* Its invariants: D pi_R P = 0 (the coarse space is projected out), and
  P^H D pi_R v = 0 (pi_L = I - D P D_c^{-1} P^H has P^H pi_L = 0).
* The solve: z = pi_R chi + P D_c^{-1} P^H b reaches its true residual, and
  agrees with the dense solution within kappa * tol."""
import numpy as np
import pytest

import oracle as O
from paper_1303_1377_amd import fields as F
from tests import _dense as DN

DIMS = (4, 4, 4, 4)
AGG = (2, 2, 2, 2)


@pytest.fixture(scope="module")
def deflated():
    U = F.make_gauge(DIMS, 0.3, 0)
    o = O.Oracle(DIMS, U, -0.2, 1.0)
    o.configure(levels=2, n_tv=[4], agg=[AGG], sap=[AGG], outer_restart=25, coarse_tol=1e-13,
                coarse_restart=60, coarse_maxit=5000)
    o.setup([F.random_vectors(256, 12, 4, 11)])
    D = DN.dense_of(o.apply, 3072)
    P = DN.dense_P(o.get_P(0), DIMS, AGG)
    Dc = P.conj().T @ D @ P
    piR = np.eye(3072) - P @ np.linalg.solve(Dc, P.conj().T @ D)
    return o, D, P, piR


def test_deflated_operator_matches_dense_product(deflated):
    o, D, P, piR = deflated
    for seed in (1, 2):
        v = F.gaussian_spinor(DIMS, seed).reshape(-1)
        got = o.apply_deflated(v).reshape(-1)
        ref = D @ (piR @ v)
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)


def test_deflated_operator_invariants(deflated):
    o, D, P, piR = deflated
    for k in (0, 5, 37):
        w = o.apply_deflated(P[:, k]).reshape(-1)
        assert np.linalg.norm(w) <= 1e-10 * np.linalg.norm(D @ P[:, k])
    v = F.gaussian_spinor(DIMS, 3).reshape(-1)
    w = o.apply_deflated(v).reshape(-1)
    assert np.linalg.norm(P.conj().T @ w) <= 1e-10 * np.linalg.norm(w)


def test_inexact_deflation_solves(deflated):
    o, D, P, piR = deflated
    b = F.gaussian_spinor(DIMS, 1000)
    x, st = o.solve_id(b, 1e-10, nu=5)
    assert st["converged"]
    assert st["true_relres"] <= 1e-9
    ex = np.linalg.solve(D, b.reshape(-1))
    kappa = np.linalg.cond(D)
    assert np.linalg.norm(x.reshape(-1) - ex) <= 2 * kappa * 1e-9 * np.linalg.norm(ex)
    r = b.reshape(-1) - D @ x.reshape(-1)
    assert abs(np.linalg.norm(r) / np.linalg.norm(b) - st["true_relres"]) <= 1e-3 * st["true_relres"] + 1e-15



def test_id_setup_update_is_the_v_cycle_from_zero():
    """IDsetup (Sec. 4.3) with n_inv = 1: after the three SAP passes the vectors
    define P and D_c, and each v_j becomes (M_SAP^(nu) pi_L + P D_c^{-1} P^H) v_j,
    normalised.  Recomputed here from dense D, the P of those vectors and the
    SAP of a second oracle instance applied to pi_L v_j."""
    U = F.make_gauge(DIMS, 0.3, 0)
    kw = dict(levels=2, n_tv=[4], agg=[AGG], sap=[AGG], nu=5, n_inv=1, coarse_tol=1e-13,
              coarse_restart=60, coarse_maxit=5000, id_setup=1)
    o = O.Oracle(DIMS, U, -0.2, 1.0)
    o.configure(**kw)
    v0 = F.random_vectors(256, 12, 4, 21)
    o.set_vectors(0, v0)
    o.setup_level(0)
    got = o.get_vectors(0).reshape(4, -1)

    ref_o = O.Oracle(DIMS, U, -0.2, 1.0)
    ref_o.configure(**kw)
    v = np.asarray(v0).reshape(4, -1).copy()
    for eta in (1, 2, 3):
        for j in range(4):
            w = ref_o.sap(0, v[j].reshape(256, 12), eta).reshape(-1)
            v[j] = w / np.linalg.norm(w)
    ref_o.set_vectors(0, v.reshape(4, 256, 12))
    ref_o.build(0)
    D = DN.dense_of(ref_o.apply, 3072)
    P = DN.dense_P(ref_o.get_P(0), DIMS, AGG)
    Dc = P.conj().T @ D @ P
    for j in range(4):
        cg = P @ np.linalg.solve(Dc, P.conj().T @ v[j])
        piL = v[j] - D @ cg
        w = ref_o.sap(0, piL.reshape(256, 12), 5).reshape(-1) + cg
        w /= np.linalg.norm(w)
        assert np.linalg.norm(got[j] - w) <= 1e-9, j
