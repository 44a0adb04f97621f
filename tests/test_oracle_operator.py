"""Pins of the oracle's Dirac operator and clover term against facts fixed by
the paper and by mathematics (not against the oracle's own formulas)."""
import numpy as np
import pytest

import oracle as O
from paper_1303_1377_amd import fields as F
from tests import _dense as DN

SMALL = (4, 2, 2, 2)


def test_gamma_algebra():
    """Sec. 2.2: Hermitian, unitary, Clifford relation, gamma5 = diag(1,1,-1,-1)."""
    g = O.gamma_matrices()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T, atol=0)
        assert np.allclose(g[mu] @ g[mu].conj().T, np.eye(4), atol=0)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2 * np.eye(4) * (mu == nu), atol=0)
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    assert np.allclose(g5, np.diag([1, 1, -1, -1]), atol=0)
    # gamma_mu gamma_nu (mu != nu) is block-diagonal in spins {0,1} / {2,3}
    for mu in range(4):
        for nu in range(4):
            if mu != nu:
                gg = g[mu] @ g[nu]
                assert np.abs(gg[:2, 2:]).max() == 0 and np.abs(gg[2:, :2]).max() == 0


@pytest.fixture(scope="module")
def small_field():
    U = F.make_gauge(SMALL, 0.3, 11)
    o = O.Oracle(SMALL, U, -0.2, 1.0)
    vol = int(np.prod(SMALL))
    D = DN.dense_of(o.apply, vol * 12)
    return U, o, D


def test_gamma5_hermiticity(small_field):
    """eq. (g5sym): (Gamma5 D)^H = Gamma5 D."""
    _, _, D = small_field
    G5 = DN.gamma5_fine(D.shape[0] // 12)
    H = G5 @ D
    assert np.abs(H - H.conj().T).max() < 1e-14


def test_spectrum_symmetric(small_field):
    """Lemma g5sym: the spectrum is closed under complex conjugation."""
    _, _, D = small_field
    ev = np.linalg.eigvals(D)
    assert DN.match_spectra(ev, np.conj(ev)) < 1e-10


def test_free_field_spectrum():
    """Unit links: plane waves diagonalise D; closed-form eigenvalues
    m0 + sum(1-cos p) +/- i sqrt(sum sin^2 p), twofold in spin, threefold in colour."""
    dims = (4, 2, 2, 2)
    m0 = -0.3
    o = O.Oracle(dims, F.unit_gauge(dims), m0, 1.7)  # clover vanishes for unit links
    D = DN.dense_of(o.apply, int(np.prod(dims)) * 12)
    ev = np.linalg.eigvals(D)
    ref = DN.free_field_eigs(dims, m0)
    assert DN.match_spectra(ev, ref) < 1e-10


def test_free_field_plane_wave_action():
    """Apply D to e^{ip.x} (x) e_(sigma,c) on a larger lattice; the result must be
    e^{ip.x} times (m0 + sum(1-cos p)) u + i sum gamma_mu sin p_mu u."""
    dims = (6, 4, 8, 2)
    m0 = 0.1
    o = O.Oracle(dims, F.unit_gauge(dims), m0, 1.0)
    g = O.gamma_matrices()
    x = DN.coords(dims)
    rng = np.random.default_rng(3)
    for _ in range(4):
        n = [rng.integers(0, d) for d in dims]
        p = np.array([2 * np.pi * n[m] / dims[m] for m in range(4)])
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * x @ p)
        psi = phase[:, None, None] * u[None]
        Mp = (m0 + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * sum(g[m] * np.sin(p[m]) for m in range(4))
        expect = phase[:, None, None] * (Mp @ u)[None]
        assert np.abs(o.apply(psi) - expect).max() < 1e-12


def test_constant_diagonal_links_spectrum():
    """Constant diagonal SU(3) links: same closed form with p_mu shifted by the
    colour phase theta_{mu c}; the clover term vanishes (abelian, constant)."""
    dims = (4, 2, 2, 2)
    m0 = -0.1
    rng = np.random.default_rng(5)
    th = rng.uniform(-np.pi, np.pi, size=(4, 2))
    theta = np.stack([th[:, 0], th[:, 1], -(th[:, 0] + th[:, 1])], axis=1)
    U = np.zeros((int(np.prod(dims)), 4, 3, 3), dtype=np.complex128)
    for mu in range(4):
        for c in range(3):
            U[:, mu, c, c] = np.exp(1j * theta[mu, c])
    o = O.Oracle(dims, U, m0, 1.0)
    D = DN.dense_of(o.apply, int(np.prod(dims)) * 12)
    ev = np.linalg.eigvals(D)
    assert DN.match_spectra(ev, DN.free_field_eigs(dims, m0, theta)) < 1e-10


def test_gauge_covariance():
    """D[U^Omega] (Omega psi) = Omega D[U] psi with U^Omega_mu(x) = Omega(x) U_mu(x) Omega(x+mu)^H
    (covers hopping terms and every clover leaf)."""
    dims = (4, 4, 2, 6)
    U = F.make_gauge(dims, 0.5, 2)
    Om = F.random_gauge_transform(dims, 9)
    x = DN.coords(dims)
    Ug = np.empty_like(U)
    for mu in range(4):
        y = x.copy()
        y[:, mu] = (y[:, mu] + 1) % dims[mu]
        j = DN.site_index(dims, y)
        Ug[:, mu] = Om @ U[:, mu] @ np.conj(np.swapaxes(Om[j], -1, -2))
    psi = F.gaussian_spinor(dims, 4)
    a = O.Oracle(dims, U, -0.3, 1.3)
    b = O.Oracle(dims, Ug, -0.3, 1.3)
    lhs = b.apply(np.einsum("xab,xsb->xsa", Om, psi))
    rhs = np.einsum("xab,xsb->xsa", Om, a.apply(psi))
    assert np.abs(lhs - rhs).max() < 1e-13 * np.abs(rhs).max() * 10


def test_clover_structure():
    """Clover term: Hermitian, traceless, chirally block diagonal; csw = 0 gives
    the Wilson operator; A(x) A(x)^{-1} = I."""
    dims = (4, 4, 4, 4)
    U = F.make_gauge(dims, 0.4, 1)
    assert O.clover_offblock(dims, U, 1.0) == 0.0
    for site in (0, 17, 255):
        T = O.clover_site(dims, U, 1.0, site)
        assert np.abs(T - T.conj().T).max() < 1e-14
        assert abs(np.trace(T)) < 1e-13
    o = O.Oracle(dims, U, -0.2, 1.0)
    A, Ai = o.clover()
    prod = np.einsum("xhij,xhjk->xhik", A, Ai)
    assert np.abs(prod - np.eye(6)).max() < 1e-12
    # csw = 0: D - D_W has no site-diagonal remainder besides (m0+4)
    w = O.Oracle(dims, U, -0.2, 0.0)
    Aw, _ = w.clover()
    assert np.abs(Aw - (3.8) * np.eye(6)).max() == 0.0


def test_clover_normalisation_constant_field():
    """Constant abelian field strength in the (1,2) plane on the torus (flux
    quantised, phase phi_c = 2 pi n_c / (N1 N2) per colour): every leaf equals
    the plaquette e^{-i phi}, so Q_12 = 4 e^{-i phi}, Q_21 = 4 e^{i phi} and the
    clover term is T = (csw/2) sin(phi_c) (i gamma_1 gamma_2) on colour c.  This
    fixes the factor csw/32, the sum over ordered (mu, nu) and the leaf
    orientation of eq. (lattice_WD)."""
    dims = (2, 4, 6, 2)
    n = np.array([1, 2, -3])
    phi = 2 * np.pi * n / (dims[1] * dims[2])
    x = DN.coords(dims)
    vol = len(x)
    U = np.zeros((vol, 4, 3, 3), dtype=np.complex128)
    for c in range(3):
        U[:, 0, c, c] = 1
        U[:, 3, c, c] = 1
        U[:, 1, c, c] = np.exp(1j * phi[c] * x[:, 2])
        top = x[:, 2] == dims[2] - 1
        U[:, 2, c, c] = np.where(top, np.exp(-1j * phi[c] * dims[2] * x[:, 1]), 1.0)
    csw = 1.3
    g = O.gamma_matrices()
    ig12 = 1j * g[1] @ g[2]
    expect = sum(np.kron(0.5 * csw * np.sin(phi[c]) * ig12, np.diag(np.eye(3)[c])) for c in range(3))
    for site in (0, 5, vol - 1, 29):
        T = O.clover_site(dims, U, csw, site)
        assert np.abs(T - expect).max() < 1e-13


def test_mass_shift_identity(small_field):
    """D(m0 + d) = D(m0) + d I."""
    U, o, D = small_field
    o2 = O.Oracle(SMALL, U, -0.2 + 0.37, 1.0)
    D2 = DN.dense_of(o2.apply, D.shape[0])
    assert np.abs(D2 - D - 0.37 * np.eye(D.shape[0])).max() < 1e-14


def test_extent_two_both_hops():
    """With extent 2 the neighbours x+mu and x-mu coincide and both hopping
    terms apply: for unit links the free-field formula still holds (checked in
    the spectrum tests); here the row sums of the hopping part equal -4 per
    direction pair times the projector sum (I-g)+(I+g) = 2I."""
    dims = (2, 2, 2, 2)
    o = O.Oracle(dims, F.unit_gauge(dims), 0.0, 1.0)
    psi = np.ones((16, 4, 3), dtype=np.complex128)
    # constant field: D psi = (m0 + 4) psi - 1/2 * sum_mu 2 psi = m0 psi = 0
    assert np.abs(o.apply(psi)).max() < 1e-14
