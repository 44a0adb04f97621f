"""Dense-matrix helpers for the oracle pins (tiny lattices only)."""
from __future__ import annotations

import numpy as np


def coords(dims):
    """Coordinates of every site in canonical order, shape (vol, 4)."""
    d = tuple(dims)
    g = np.indices(d).reshape(4, -1).T
    return g


def site_index(dims, x):
    x = np.asarray(x)
    return ((x[..., 0] * dims[1] + x[..., 1]) * dims[2] + x[..., 2]) * dims[3] + x[..., 3]


def dense_of(apply, n, dtype=np.complex128):
    """Dense matrix of a linear map given as a callable on flat vectors."""
    m = np.zeros((n, n), dtype=dtype)
    e = np.zeros(n, dtype=dtype)
    for i in range(n):
        e[:] = 0
        e[i] = 1
        m[:, i] = np.asarray(apply(e)).reshape(n)
    return m


def gamma5_fine(vol):
    return np.kron(np.eye(vol), np.kron(np.diag([1.0, 1.0, -1.0, -1.0]), np.eye(3)))


def gamma5_coarse(volc, nv):
    return np.kron(np.eye(volc), np.diag(np.r_[np.ones(nv), -np.ones(nv)]))


def aggregate_index(dims, agg):
    """Coarse site of every fine site for lattice blocks of size agg."""
    x = coords(dims)
    cd = [dims[m] // agg[m] for m in range(4)]
    bc = x // np.asarray(agg)
    return site_index(cd, bc), tuple(cd)


def dense_P(P, dims, agg):
    """Dense interpolation matrix from columns P[k][x][d] (d < nd/2: half 0)."""
    nv, vol, nd = P.shape
    ai, cd = aggregate_index(dims, agg)
    volc = int(np.prod(cd))
    out = np.zeros((vol * nd, volc * 2 * nv), dtype=np.complex128)
    h0 = nd // 2
    for x in range(vol):
        for d in range(nd):
            for k in range(nv):
                out[x * nd + d, ai[x] * 2 * nv + (d // h0) * nv + k] = P[k, x, d]
    return out


def dense_coarse(M, cdims):
    """Dense coarse operator from stencil blocks M[c][slot][a][b]."""
    volc, _, n, _ = M.shape
    x = coords(cdims)
    out = np.zeros((volc * n, volc * n), dtype=np.complex128)
    for c in range(volc):
        out[c * n:(c + 1) * n, c * n:(c + 1) * n] += M[c, 0]
        for mu in range(4):
            for sgn, slot in ((1, 1 + mu), (-1, 5 + mu)):
                y = x[c].copy()
                y[mu] = (y[mu] + sgn) % cdims[mu]
                j = site_index(cdims, y)
                out[c * n:(c + 1) * n, j * n:(j + 1) * n] += M[c, slot]
    return out


def block_masks(dims, b):
    """Block id and colour (even sum of block coordinates = 0) of every site."""
    x = coords(dims)
    nbk = [dims[m] // b[m] for m in range(4)]
    bc = x // np.asarray(b)
    bid = site_index(nbk, bc)
    col = bc.sum(axis=1) % 2
    return bid, col


def free_field_eigs(dims, m0, theta=None):
    """Closed-form spectrum of D for unit links (theta=None) or for constant
    diagonal links with colour phases theta[mu][c]:  for each momentum p with
    p_mu = 2 pi n_mu / N_mu (shifted by theta per colour),
        lambda = m0 + sum_mu (1 - cos p_mu) +/- i sqrt(sum_mu sin^2 p_mu),
    each sign twofold in spin."""
    ev = []
    ranges = [np.arange(n) * 2 * np.pi / n for n in dims]
    for n0 in ranges[0]:
        for n1 in ranges[1]:
            for n2 in ranges[2]:
                for n3 in ranges[3]:
                    p = np.array([n0, n1, n2, n3])
                    for c in range(3):
                        q = p if theta is None else p + np.array([theta[m][c] for m in range(4)])
                        re = m0 + np.sum(1 - np.cos(q))
                        im = np.sqrt(np.sum(np.sin(q) ** 2))
                        ev += [re + 1j * im, re + 1j * im, re - 1j * im, re - 1j * im]
    return np.array(ev)


def match_spectra(a, b):
    """Max distance between two eigenvalue multisets (greedy nearest matching)."""
    a = list(np.asarray(a))
    b = list(np.asarray(b))
    assert len(a) == len(b)
    worst = 0.0
    b_arr = np.array(b)
    used = np.zeros(len(b), dtype=bool)
    for v in a:
        d = np.abs(b_arr - v)
        d[used] = np.inf
        j = int(np.argmin(d))
        used[j] = True
        worst = max(worst, float(d[j]))
    return worst
