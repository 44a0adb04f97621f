"""The device-side link generator (used where host generation is too slow)
follows the host recipe: on the same random draw its exp(i eps H) matches the
eigen-decomposition form, and its APE steps (Newton polar projection) match
the host's (SVD polar projection) to rounding; the links are SU(3)."""
import numpy as np
import pytest

from paper_1303_1377_amd import fields as F

torch = pytest.importorskip("torch")


def _draw(n, eps, seed):
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    re = torch.randn((n, 3, 3), generator=g, dtype=torch.float64)
    im = torch.randn((n, 3, 3), generator=g, dtype=torch.float64)
    a = (re + 1j * im).numpy()
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1).real / 3.0
    h = h - tr[..., None, None] * np.eye(3)
    lam, vec = np.linalg.eigh(h)
    return F.reunitarise(np.einsum("...ij,...j,...kj->...ik", vec, np.exp(1j * eps * lam), np.conj(vec)))


def test_device_generator_follows_host_recipe():
    dims = (4, 2, 4, 4)
    n = 4 * int(np.prod(dims))
    u0 = F.make_gauge_device(dims, 0.4, 3, ape_steps=0, device="cpu", chunk=n).numpy()
    assert np.abs(u0.reshape(n, 3, 3) - _draw(n, 0.4, 3)).max() < 1e-13
    u2 = F.make_gauge_device(dims, 0.4, 3, ape_steps=2, device="cpu", chunk=n).numpy()
    ref = F.ape_smear(F.ape_smear(u0.reshape(dims + (4, 3, 3)), 0.5), 0.5).reshape(u2.shape)
    assert np.abs(u2 - ref).max() < 1e-13
    ident = np.einsum("...ij,...kj->...ik", u2, u2.conj())
    assert np.abs(ident - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(u2) - 1.0).max() < 1e-13
