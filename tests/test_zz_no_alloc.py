"""The allocation-free stencil entry point dd_apply_D_noalloc (fixed device
staging array instead of per-call allocations) against dd_apply, which runs the
same kernels on freshly allocated staging buffers: two and more calls in a row,
the later ones on smaller lattices, so that each call must overwrite what the
previous one left in the shared array."""
import numpy as np
import pytest

from tests._gpu import rel, say, to_np

pytestmark = pytest.mark.gpu


def _one(dims, seed):
    import torch

    import oracle as O
    import paper_1303_1377_amd as G
    from paper_1303_1377_amd import fields as F

    say("no-alloc D apply: dims %s seed %d" % (dims, seed))
    U = F.make_gauge(dims, 0.3, seed)
    s = G.Solver(dims, U, -0.2, 1.0)
    psi = F.gaussian_spinor(dims, 100 + seed)
    ref, _ = s.apply("D", 0, psi)
    out = torch.full_like(ref, float("nan"))
    s.apply_D_noalloc(psi, out=out)
    torch.cuda.synchronize()
    a, b = to_np(out), to_np(ref)
    assert np.isfinite(a).all()
    err = rel(a, b)
    say("  vs dd_apply: %.3e" % err)
    assert err <= 1e-13, err
    if np.prod(dims) <= 4096:
        eo = rel(a, O.Oracle(dims, U, -0.2, 1.0).apply(psi))
        say("  vs oracle: %.3e" % eo)
        assert eo <= 1e-13, eo
    s.close()


def test_noalloc_equals_dd_apply_on_shrinking_lattices():
    """16^4 (the largest lattice the fixed array holds), then 8^4, then 4^4."""
    _one((16, 16, 16, 16), 1)
    _one((8, 8, 8, 8), 2)
    _one((4, 4, 4, 4), 3)


def test_noalloc_rejects_lattices_above_the_limit():
    import paper_1303_1377_amd as G
    from paper_1303_1377_amd import fields as F

    dims = (20, 16, 16, 16)   # 81,920 sites > 65,536
    say("no-alloc D apply: limit check at %s" % (dims,))
    s = G.Solver(dims, F.unit_gauge(dims), 0.1, 1.0)
    with pytest.raises(G.DDError) as ei:
        s.apply_D_noalloc(F.gaussian_spinor(dims, 1))
    assert ei.value.code == -1 and "allocation-free limit" in str(ei.value)
    s.close()
