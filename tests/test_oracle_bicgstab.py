"""Pins of the oracle's comparison solver (Sec. 6): odd-even preconditioned
BiCGStab, and FGMRES right-preconditioned by a fixed number of its steps.

* The odd-even reduction: whatever the number of BiCGStab steps, the
  back-substituted x makes the residual b - D x vanish on the even sites.
* The exact limit: enough steps solve the reduced system, so x equals the
  dense direct solution D^{-1} b (2^4 and 4^4).
* The outer solve reaches its true residual and agrees with the dense
  solution within kappa * tol."""
import numpy as np

import oracle as O
from paper_1303_1377_amd import fields as F
from tests import _dense as DN


def _even_rows(dims):
    x = DN.coords(dims)
    par = x.sum(axis=1) % 2
    return np.concatenate([np.arange(12 * s, 12 * s + 12) for s in np.where(par == 0)[0]])


def test_back_substitution_zeroes_the_even_residual():
    dims = (4, 4, 2, 2)
    U = F.make_gauge(dims, 0.35, 2)
    o = O.Oracle(dims, U, -0.1, 1.0)
    D = DN.dense_of(o.apply, 64 * 12)
    b = F.gaussian_spinor(dims, 3).reshape(-1)
    ev = _even_rows(dims)
    for steps in (1, 3, 7):
        x, its = o.bicgstab(b, steps)
        assert its == steps
        r = b - D @ x.reshape(-1)
        assert np.abs(r[ev]).max() < 1e-13 * np.abs(b).max()
        assert np.linalg.norm(r) < np.linalg.norm(b)


def test_many_steps_give_the_dense_solution():
    for dims, m0, steps in (((2, 2, 2, 2), -0.2, 150), ((4, 4, 4, 4), 0.1, 300)):
        U = F.make_gauge(dims, 0.3, 0)
        o = O.Oracle(dims, U, m0, 1.0)
        n = int(np.prod(dims)) * 12
        D = DN.dense_of(o.apply, n)
        b = F.gaussian_spinor(dims, 7).reshape(-1)
        x, its = o.bicgstab(b, steps)
        ex = np.linalg.solve(D, b)
        assert np.linalg.norm(x.reshape(-1) - ex) < 1e-9 * np.linalg.norm(ex), dims


def test_fgmres_with_bicgstab_preconditioner_solves():
    dims = (4, 4, 4, 4)
    U = F.make_gauge(dims, 0.3, 0)
    o = O.Oracle(dims, U, -0.2, 1.0)
    o.configure(levels=2, n_tv=[4], agg=[(2, 2, 2, 2)], sap=[(2, 2, 2, 2)], outer_restart=25)
    b = F.gaussian_spinor(dims, 1000)
    x, st = o.solve_bicgstab(b, 1e-10, 50)
    assert st["converged"] and st["true_relres"] <= 1e-10
    D = DN.dense_of(o.apply, 3072)
    ex = np.linalg.solve(D, b.reshape(-1))
    kappa = np.linalg.cond(D)
    assert np.linalg.norm(x.reshape(-1) - ex) <= 2 * kappa * 1e-10 * np.linalg.norm(ex)
