"""The Krylov-Schur eigenvalue routine that fixes the workloads' masses
(m0 = m_crit + shift, m_crit = -Re lambda_SR(D(m0 = 0))), run on the CPU with
the oracle's operator, against dense eigenvalues of the same operator."""
import numpy as np

import oracle as O
from paper_1303_1377_amd import fields as F
from paper_1303_1377_amd.mcrit import smallest_real_eigs
from tests import _dense as DN


def test_krylov_schur_smallest_real_part_matches_dense():
    import torch

    dims = (4, 4, 2, 2)
    U = F.make_gauge(dims, 0.4, 1, ape_steps=2, ape_alpha=0.5)
    o = O.Oracle(dims, U, 0.0, 1.0)
    n = int(np.prod(dims)) * 12
    ev_dense = np.linalg.eigvals(DN.dense_of(o.apply, n))
    ev_dense = ev_dense[np.argsort(ev_dense.real)]

    def apply(v):
        return torch.as_tensor(o.apply(v.numpy()))

    ev, res, mv, rs = smallest_real_eigs(apply, n, nev=3, m=30, tol=1e-10, device="cpu")
    assert np.all(res <= 1e-10)
    assert abs(ev[0].real - ev_dense[0].real) < 1e-8
    # the three smallest real parts (conjugate pairs share theirs)
    assert np.abs(np.sort(ev.real) - ev_dense[:3].real).max() < 1e-7
