"""Seeded synthetic inputs: gauge configurations, right-hand sides, test vectors.

This module only draws random numbers and builds SU(3) link fields; it holds
none of the solver's arithmetic (no Dirac operator, no smoother, no multigrid).
Both the HIP path and the CPU oracle take their inputs from here.

Conventions (paper Sec. 2.2, lattice definition and spinor index order):
  * lattice dims are (N0, N1, N2, N3) with x0 the time direction;
  * canonical site index  ((x0*N1 + x1)*N2 + x2)*N3 + x3;
  * spinor layout [site][spin 0..3][colour 0..2], colour fastest;
  * gauge layout  [site][mu 0..3][row][col], U_mu(x) on the link x -> x+mu.

Link generator (synthetic stand-in for the paper's production ensembles of
Table 2, which are not available): U = exp(i*eps*H) with H traceless
Hermitian built from complex N(0,1) entries, reunitarised to SU(3);
optionally followed by APE smearing steps projected back to SU(3).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "lattice_volume",
    "random_su3",
    "reunitarise",
    "project_su3",
    "ape_smear",
    "make_gauge",
    "gaussian_spinor",
    "point_source",
    "random_vectors",
    "random_gauge_transform",
    "unit_gauge",
]


def lattice_volume(dims) -> int:
    d = [int(v) for v in dims]
    return d[0] * d[1] * d[2] * d[3]


def _cgauss(rng: np.random.Generator, shape) -> np.ndarray:
    """Complex normal numbers: real and imaginary parts i.i.d. N(0,1)."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return re + 1j * im


def reunitarise(u: np.ndarray) -> np.ndarray:
    """Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1): exact SU(3)."""
    u = np.array(u, dtype=np.complex128, copy=True)
    r0 = u[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    out = np.empty_like(u)
    out[..., 0, :] = r0
    out[..., 1, :] = r1
    out[..., 2, :] = r2
    return out


def random_su3(shape, eps: float, rng: np.random.Generator) -> np.ndarray:
    """SU(3) matrices exp(i*eps*H), H traceless Hermitian from N(0,1) entries."""
    a = _cgauss(rng, tuple(shape) + (3, 3))
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h = h - tr[..., None, None] * np.eye(3)
    lam, vec = np.linalg.eigh(h)
    ph = np.exp(1j * eps * lam)
    u = np.einsum("...ij,...j,...kj->...ik", vec, ph, np.conj(vec))
    return reunitarise(u)


def project_su3(w: np.ndarray) -> np.ndarray:
    """Nearest unitary matrix (polar factor via SVD), phase fixed to det = 1."""
    x, _, yh = np.linalg.svd(w)
    u = x @ yh
    det = np.linalg.det(u)
    u = u * np.exp(-1j * np.angle(det) / 3.0)[..., None, None]
    return reunitarise(u)


def _shift(u: np.ndarray, mu: int, step: int) -> np.ndarray:
    """Field value at x + step*mu (periodic); u has the 4 lattice axes first."""
    return np.roll(u, -step, axis=mu)


def _dag(m: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(m, -1, -2))


def ape_smear(u: np.ndarray, alpha: float) -> np.ndarray:
    """One APE smearing step on a (N0,N1,N2,N3,4,3,3) field, all links at once.

    V_mu = (1-alpha) U_mu + alpha/6 * sum_{nu != mu} (upper + lower staples),
    then projected back to SU(3).
    """
    out = np.empty_like(u)
    for mu in range(4):
        umu = u[..., mu, :, :]
        staple = np.zeros_like(umu)
        for nu in range(4):
            if nu == mu:
                continue
            unu = u[..., nu, :, :]
            # U_nu(x) U_mu(x+nu) U_nu(x+mu)^H
            staple += unu @ _shift(umu, nu, 1) @ _dag(_shift(unu, mu, 1))
            # U_nu(x-nu)^H U_mu(x-nu) U_nu(x-nu+mu)
            unu_m = _shift(unu, nu, -1)
            staple += _dag(unu_m) @ _shift(umu, nu, -1) @ _shift(_shift(unu, nu, -1), mu, 1)
        out[..., mu, :, :] = project_su3((1.0 - alpha) * umu + (alpha / 6.0) * staple)
    return out


def make_gauge(dims, eps: float, seed: int, ape_steps: int = 0, ape_alpha: float = 0.5) -> np.ndarray:
    """Seeded SU(3) gauge field, returned flat as [site][mu][3][3] complex128."""
    d = tuple(int(v) for v in dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    u = random_su3(d + (4,), eps, rng)
    for _ in range(ape_steps):
        u = ape_smear(u, ape_alpha)
    return np.ascontiguousarray(u.reshape(lattice_volume(d), 4, 3, 3))


def unit_gauge(dims) -> np.ndarray:
    v = lattice_volume(dims)
    u = np.zeros((v, 4, 3, 3), dtype=np.complex128)
    u[:, :, 0, 0] = u[:, :, 1, 1] = u[:, :, 2, 2] = 1.0
    return u


def random_gauge_transform(dims, seed: int) -> np.ndarray:
    """Site-local SU(3) matrices Omega(x), flat [site][3][3]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return random_su3((lattice_volume(dims),), 1.0, rng)


def gaussian_spinor(dims, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Complex N(0,1) spinor field(s): [site][4][3] or [nrhs][site][4][3]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = lattice_volume(dims)
    shape = (v, 4, 3) if nrhs is None else (nrhs, v, 4, 3)
    return np.ascontiguousarray(_cgauss(rng, shape))


def point_source(dims, site: int, spin: int, colour: int) -> np.ndarray:
    b = np.zeros((lattice_volume(dims), 4, 3), dtype=np.complex128)
    b[site, spin, colour] = 1.0
    return b


def random_vectors(n_sites: int, nd: int, count: int, seed: int) -> np.ndarray:
    """Initial test vectors for the adaptive setup: [count][n_sites][nd], complex N(0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(_cgauss(rng, (count, n_sites, nd)))
