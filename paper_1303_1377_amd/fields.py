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
    "make_gauge_device",
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


# ---------------------------------------------------------------------------
# The same link recipe drawn on the GPU, for lattices whose host generation
# would take too long (tens of millions of links).  The random stream is
# torch's Philox generator on the device, so the field is a different draw
# from make_gauge with the same seed; the distribution and the steps are the
# same: exp(i eps H) (Taylor series with scaling and squaring), reunitarised,
# then APE steps with the polar projection (Newton iteration
# X <- (X + X^-H)/2, then det phase and reunitarisation).  3x3 products are written out element-wise (no batched
# BLAS calls).  Returns a [site][mu][3][3] complex128 tensor on the device.
# ---------------------------------------------------------------------------
def _t_mm(a, b):
    return (a.unsqueeze(-1) * b.unsqueeze(-3)).sum(-2)


def _t_dag(a):
    return a.transpose(-1, -2).conj()


def _t_det(a):
    return (a[..., 0, 0] * (a[..., 1, 1] * a[..., 2, 2] - a[..., 1, 2] * a[..., 2, 1])
            - a[..., 0, 1] * (a[..., 1, 0] * a[..., 2, 2] - a[..., 1, 2] * a[..., 2, 0])
            + a[..., 0, 2] * (a[..., 1, 0] * a[..., 2, 1] - a[..., 1, 1] * a[..., 2, 0]))


def _t_inv(a):
    import torch

    c = torch.empty_like(a)
    for i in range(3):
        for j in range(3):
            r = [q for q in range(3) if q != j]
            s = [q for q in range(3) if q != i]
            m = a[..., r[0], s[0]] * a[..., r[1], s[1]] - a[..., r[0], s[1]] * a[..., r[1], s[0]]
            c[..., i, j] = m if (i + j) % 2 == 0 else -m
    return c / _t_det(a)[..., None, None]


def _t_reunitarise(u):
    import torch

    r0 = u[..., 0, :]
    r0 = r0 / torch.linalg.vector_norm(r0, dim=-1, keepdim=True)
    r1 = u[..., 1, :]
    r1 = r1 - (r0.conj() * r1).sum(-1, keepdim=True) * r0
    r1 = r1 / torch.linalg.vector_norm(r1, dim=-1, keepdim=True)
    r2 = torch.stack([r0[..., 1] * r1[..., 2] - r0[..., 2] * r1[..., 1],
                      r0[..., 2] * r1[..., 0] - r0[..., 0] * r1[..., 2],
                      r0[..., 0] * r1[..., 1] - r0[..., 1] * r1[..., 0]], dim=-1).conj()
    return torch.stack([r0, r1, r2], dim=-2)


def _t_project(w, iters=12):
    import torch

    x = w
    for _ in range(iters):
        x = 0.5 * (x + _t_dag(_t_inv(x)))
    ph = torch.exp(-1j * torch.angle(_t_det(x)) / 3.0)
    return _t_reunitarise(x * ph[..., None, None])


def _t_random_su3(n, eps, gen, device):
    import torch

    re = torch.randn((n, 3, 3), generator=gen, device=device, dtype=torch.float64)
    im = torch.randn((n, 3, 3), generator=gen, device=device, dtype=torch.float64)
    a = torch.complex(re, im)
    del re, im
    h = 0.5 * (a + _t_dag(a))
    tr = (h[..., 0, 0] + h[..., 1, 1] + h[..., 2, 2]).real / 3.0
    for q in range(3):
        h[..., q, q] -= tr
    # exp(i eps H): Taylor series of degree 14 on A / 2^5, then 5 squarings
    a = (1j * eps / 32.0) * h
    u = torch.zeros_like(a)
    term = torch.zeros_like(a)
    for q in range(3):
        u[..., q, q] = 1.0
        term[..., q, q] = 1.0
    for k in range(1, 15):
        term = _t_mm(term, a) / k
        u = u + term
    for _ in range(5):
        u = _t_mm(u, u)
    return _t_reunitarise(u)


def make_gauge_device(dims, eps: float, seed: int, ape_steps: int = 0, ape_alpha: float = 0.5, device="cuda",
                      chunk: int = 1 << 21, log=None):
    """The make_gauge recipe on the GPU (see above): [site][mu][3][3] complex128."""
    import torch

    d = tuple(int(v) for v in dims)
    vol = lattice_volume(d)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    u = torch.empty((vol * 4, 3, 3), dtype=torch.complex128, device=device)
    for s in range(0, vol * 4, chunk):
        e = min(vol * 4, s + chunk)
        u[s:e] = _t_random_su3(e - s, eps, gen, device)
    u = u.reshape(d + (4, 3, 3))
    if log:
        log("make_gauge_device: SU(3) links drawn")
    for step in range(ape_steps):
        out = torch.empty_like(u)
        for mu in range(4):
            umu = u[..., mu, :, :]
            staple = torch.zeros_like(umu)
            for nu in range(4):
                if nu == mu:
                    continue
                unu = u[..., nu, :, :]
                # U_nu(x) U_mu(x+nu) U_nu(x+mu)^H
                staple += _t_mm(_t_mm(unu, torch.roll(umu, -1, nu)), _t_dag(torch.roll(unu, -1, mu)))
                # U_nu(x-nu)^H U_mu(x-nu) U_nu(x-nu+mu)
                unu_m = torch.roll(unu, 1, nu)
                staple += _t_mm(_t_mm(_t_dag(unu_m), torch.roll(umu, 1, nu)), torch.roll(unu_m, -1, mu))
                del unu_m
            out[..., mu, :, :] = _t_project((1.0 - ape_alpha) * umu + (ape_alpha / 6.0) * staple)
            del staple
        u = out
        if log:
            log("make_gauge_device: APE step %d done" % (step + 1))
    return u.reshape(vol, 4, 3, 3)
