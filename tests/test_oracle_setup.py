"""Pins of the oracle's adaptive setup (Algorithm 2) and of its mass shift.

The setup is an iteration with no closed form, but with exact block solves
(many MR steps) every step of it is a map that dense linear algebra can write
out on a tiny lattice:

  * the three initial passes  v <- M_SAP^(eta) v,  eta = 1, 2, 3, with
    M_SAP^(eta) = sum_{k<eta} (I - K D)^k K and K = B_black (I - D B_red) + B_red
    (Sec. 2.3);
  * each of the n_inv rounds builds P by a QR with positive diagonal per
    aggregate and chirality half (Sec. 3.1, standard aggregation) and
    D_c = P^H D P, then updates every vector by  v <- v + C (v - D v)  with the
    V-cycle  C = M_SAP^(nu) pi_L + P D_c^{-1} P^H  (eq. iterationmatrix,
    Algorithm 2) and normalises it (Algorithm 1);
  * P and D_c are rebuilt once more from the final vectors.

The coarse solve is either exact (tiny tolerance) or a fixed number k of
odd-even GMRES steps (Sec. 5), written from GMRES's definition: the odd-site
Schur system S e_o = f_o is solved by the minimiser of the residual over the
Krylov space K_k(S, f_o), and the even sites follow by back-substitution.  With
an exact coarse solve Algorithm 2's update equals Algorithm 1's (the test
vectors lie in range(P), which the exact coarse-grid correction removes from
v - D v), so only the inexact case tells them apart.

The dense side below is written from those formulas with numpy's QR, inverse
and solve; it shares nothing with the oracle except the matrix of D, which the
operator pins (closed-form spectra, gauge covariance, Gamma5-hermiticity) fix.
"""
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
M0 = 0.3


def _oracle(n_inv, coarse_k=None, nu=2, m0=M0, seed=3):
    U = F.make_gauge(DIMS, 0.35, seed)
    o = O.Oracle(DIMS, U, m0, 1.0)
    if coarse_k is None:
        ckw = dict(coarse_tol=1e-15, coarse_restart=64, coarse_maxit=5000)
    else:
        ckw = dict(coarse_fixed=coarse_k, coarse_restart=30)
    o.configure(levels=2, n_tv=[NV], agg=[AGG], sap=[SAPB], mr_steps=[400], nu=nu, n_inv=n_inv, **ckw)
    return U, o


def _sap_K(D):
    """Dense red-black SAP with exact block inverses: K and E = I - K D."""
    n = D.shape[0]
    bid, col = DN.block_masks(DIMS, SAPB)
    B = [np.zeros((n, n), dtype=np.complex128) for _ in range(2)]
    for b in np.unique(bid):
        sites = np.where(bid == b)[0]
        idx = np.concatenate([np.arange(12 * s, 12 * s + 12) for s in sites])
        B[col[sites[0]]][np.ix_(idx, idx)] += np.linalg.inv(D[np.ix_(idx, idx)])
    K = B[1] @ (np.eye(n) - D @ B[0]) + B[0]
    return K, np.eye(n) - K @ D


def _M_sap(K, E, eta):
    return sum(np.linalg.matrix_power(E, k) for k in range(eta)) @ K


def _columns_qr(V):
    """Interpolation columns [N][vol][12] from test vectors [N][vol][12]: for
    every aggregate and chirality half the thin QR of [v_1 .. v_N] with a
    positive real diagonal of R (Gram-Schmidt in the order v_1 .. v_N)."""
    ai, cd = DN.aggregate_index(DIMS, AGG)
    out = np.zeros_like(V)
    for a in range(int(np.prod(cd))):
        sites = np.where(ai == a)[0]
        for h in range(2):
            W = np.stack([V[k][sites][:, 6 * h:6 * h + 6].reshape(-1) for k in range(NV)], axis=1)
            Q, R = np.linalg.qr(W)
            ph = np.diag(R) / np.abs(np.diag(R))
            Q = Q * ph[None, :]
            for k in range(NV):
                out[k][np.ix_(sites, np.arange(6 * h, 6 * h + 6))] = Q[:, k].reshape(len(sites), 6)
    return out


def _coarse_parity(ndc):
    xc = DN.coords(tuple(DIMS[m] // AGG[m] for m in range(4)))
    par = np.repeat(xc.sum(axis=1) % 2, ndc)
    return np.where(par == 0)[0], np.where(par == 1)[0]


def _coarse_solve(Dc, r, k):
    """Coarse solve: exact (k None) or k odd-even GMRES steps from zero."""
    if k is None:
        return np.linalg.solve(Dc, r)
    ev, od = _coarse_parity(2 * NV)
    Aee = Dc[np.ix_(ev, ev)]
    S = Dc[np.ix_(od, od)] - Dc[np.ix_(od, ev)] @ np.linalg.solve(Aee, Dc[np.ix_(ev, od)])
    f = r[od] - Dc[np.ix_(od, ev)] @ np.linalg.solve(Aee, r[ev])
    cols = [f]
    for _ in range(k - 1):
        cols.append(S @ cols[-1])
    Q, _ = np.linalg.qr(np.stack(cols, axis=1))
    y = np.linalg.lstsq(S @ Q, f, rcond=None)[0]
    e = np.zeros_like(r)
    e[od] = Q @ y
    e[ev] = np.linalg.solve(Aee, r[ev] - Dc[np.ix_(ev, od)] @ e[od])
    return e


def _vcycle(D, K, E, P, Dc, r, k, nu):
    """No pre-smoothing, coarse correction, nu SAP iterations (Sec. 4.2)."""
    z = P @ _coarse_solve(Dc, P.conj().T @ r, k)
    for _ in range(nu):
        z = z + K @ (r - D @ z)
    return z


def _dense_setup(D, v0, n_inv, coarse_k=None, nu=2, update="alg2"):
    """Algorithm 2 written densely (exact block solves)."""
    K, E = _sap_K(D)
    V = [v.reshape(-1).copy() for v in v0]
    for eta in (1, 2, 3):
        Me = _M_sap(K, E, eta)
        V = [Me @ v for v in V]
        V = [v / np.linalg.norm(v) for v in V]
    for _ in range(n_inv):
        P = DN.dense_P(_columns_qr(np.stack(V).reshape(NV, VOL, 12)), DIMS, AGG)
        Dc = P.conj().T @ D @ P
        if update == "alg2":
            V = [v + _vcycle(D, K, E, P, Dc, v - D @ v, coarse_k, nu) for v in V]
        else:
            V = [_vcycle(D, K, E, P, Dc, v, coarse_k, nu) for v in V]
        V = [v / np.linalg.norm(v) for v in V]
    Vf = np.stack(V).reshape(NV, VOL, 12)
    Pc = _columns_qr(Vf)
    P = DN.dense_P(Pc, DIMS, AGG)
    return Vf, Pc, P.conj().T @ D @ P


@pytest.mark.parametrize("n_inv,coarse_k", [(0, None), (1, None), (2, None), (1, 3), (2, 3)])
def test_setup_algorithm2_equals_dense(n_inv, coarse_k):
    """Algorithm 2 (with the readings: normalise after each initial pass,
    rebuild P and D_c from the final vectors) against its dense form.  A
    mistake in the update (Algorithm 1's C v instead of v + C(v - D v)), a
    missing normalisation or a missing final rebuild changes the vectors, P or
    D_c by O(1)."""
    U, o = _oracle(n_inv, coarse_k)
    v0 = F.random_vectors(VOL, 12, NV, 77)
    o.set_vectors(0, v0)
    o.setup_level(0)
    D = DN.dense_of(o.apply, VOL * 12)
    Vd, Pd, Dcd = _dense_setup(D, v0, n_inv, coarse_k)
    Vo = o.get_vectors(0)
    Po = o.get_P(0)
    cd, _ = o.level_info(1)
    Dco = DN.dense_coarse(o.get_coarse(1)[0], cd)
    ev = np.abs(Vo - Vd).max() / np.abs(Vd).max()
    ep = np.abs(Po - Pd).max() / np.abs(Pd).max()
    ec = np.abs(Dco - Dcd).max() / np.abs(Dcd).max()
    assert ev < 1e-10 and ep < 1e-10 and ec < 1e-10, (ev, ep, ec)
    for v in Vo:
        assert abs(np.linalg.norm(v) - 1.0) < 1e-13


def test_setup_update_differs_from_inexact_deflation():
    """Sanity of the pin above: with an inexact (3-step) coarse solve,
    Algorithm 1's update C v gives vectors different from Algorithm 2's
    v + C(v - D v), so the comparison above tells the two apart; with an
    exact coarse solve both updates agree (v lies in range(P))."""
    U, o = _oracle(1, 3)
    v0 = F.random_vectors(VOL, 12, NV, 77)
    D = DN.dense_of(o.apply, VOL * 12)
    V2, _, _ = _dense_setup(D, v0, 2, 3)
    V1, _, _ = _dense_setup(D, v0, 2, 3, update="alg1")
    assert np.abs(V1 - V2).max() > 1e-4 * np.abs(V2).max()
    V2, _, _ = _dense_setup(D, v0, 1, None)
    V1, _, _ = _dense_setup(D, v0, 1, None, update="alg1")
    assert np.abs(V1 - V2).max() < 1e-10


def test_shift_mass_equals_fresh_context():
    """Changing m0 on a context (A -> A + dm I, inverses recomputed) gives the
    operator and the clover blocks of a context created at m0 + dm (the mass
    enters D only through the diagonal (m0 + 4) I of eq. lattice_WD)."""
    U = F.make_gauge(DIMS, 0.35, 5)
    dm = 0.137
    o1 = O.Oracle(DIMS, U, -0.2, 1.0)
    o1.shift_mass(dm)
    o2 = O.Oracle(DIMS, U, -0.2 + dm, 1.0)
    A1, Ai1 = o1.clover()
    A2, Ai2 = o2.clover()
    assert np.abs(A1 - A2).max() < 1e-14
    assert np.abs(Ai1 - Ai2).max() < 1e-13 * np.abs(Ai2).max()
    for x in range(VOL):
        for h in range(2):
            assert np.abs(A1[x, h] @ Ai1[x, h] - np.eye(6)).max() < 1e-13
    psi = F.gaussian_spinor(DIMS, 9)
    y1, y2 = o1.apply(psi), o2.apply(psi)
    assert np.abs(y1 - y2).max() < 1e-14 * np.abs(y2).max()
    # and exactly D(m0 + dm) = D(m0) + dm I
    o0 = O.Oracle(DIMS, U, -0.2, 1.0)
    assert np.abs(y1 - o0.apply(psi) - dm * psi).max() < 1e-13 * np.abs(y1).max()
