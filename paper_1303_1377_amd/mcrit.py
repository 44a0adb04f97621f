"""Critical mass of a generated gauge field.

The workloads fix their bare mass relative to the critical mass of their own
field: m0 = m_crit + shift with m_crit = -Re lambda_SR(D(m0 = 0)), lambda_SR the
eigenvalue of smallest real part of the clover-Wilson operator at zero mass
(the mass enters D only through (m0 + 4) I, so D(m0) = D(0) + m0 I and
m0 = m_crit makes the left edge of the spectrum touch the imaginary axis).

`smallest_real_eigs` is a Krylov-Schur iteration (thick-restart Arnoldi,
G. W. Stewart, SIAM J. Matrix Anal. Appl. 23 (2001)): Arnoldi with classical
Gram-Schmidt and one re-orthogonalisation up to m vectors, a Schur form of the
small Hessenberg matrix with the `keep` Ritz values of smallest real part moved
to the front, truncation to those, continuation.  The basis lives on the
device as torch tensors; the operator is any callable on flat complex128
vectors.  `m_crit` drives it with the library's FP64 stencil (dd_apply),
which is how the masses of lattices too large for the CPU oracle are fixed.

    python -m paper_1303_1377_amd.mcrit --dims 96,48,48,48 --eps 0.4 --ape 2 --seed 0 [--device-field]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def smallest_real_eigs(apply, n, nev=4, m=64, keep=None, tol=1e-8, max_restarts=400, seed=0, device="cuda",
                       log=None, max_seconds=None):
    """Eigenvalues of smallest real part of the operator `apply` (flat complex128
    tensor of length n -> same).  Returns (eigenvalues sorted by real part,
    relative residual estimates, matvec count, restart count); converged when
    the residual estimate |h_{m+1,m} y_m| of each of the nev wanted Ritz pairs
    is at most tol * |theta|, or after max_restarts restarts or max_seconds
    (the estimates are then returned with their residuals).  Near the left
    edge of a large lattice's spectrum the eigenvalues cluster: a basis of 64
    vectors converged where one of 40 stagnated."""
    t_start = time.time()
    import scipy.linalg as sla
    import torch

    keep = keep or max(nev + 2, m // 2)
    assert nev <= keep < m
    g = torch.Generator(device="cpu").manual_seed(seed)
    V = torch.empty((m + 1, n), dtype=torch.complex128, device=device)
    v0 = torch.complex(torch.randn(n, generator=g, dtype=torch.float64), torch.randn(n, generator=g, dtype=torch.float64))
    V[0] = v0.to(device) / torch.linalg.vector_norm(v0)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    k = 0            # basis vectors already orthonormal (and H[:k+1, :k] valid)
    matvecs = 0
    chunk = max(1, (1 << 27) // max(m, 1))   # columns per block of the in-place basis rotation
    for restart in range(max_restarts + 1):
        for j in range(k, m):
            w = apply(V[j])
            matvecs += 1
            h = torch.zeros(j + 1, dtype=torch.complex128, device=device)
            Vr = torch.view_as_real(V[: j + 1]).reshape(j + 1, 2 * n)
            for _ in range(2):   # CGS with one re-orthogonalisation
                # V^H w as two real matrix-vector products on the interleaved
                # (re, im) view: Re = Vr (x, y), Im = Vr (y, -x) for w = x + i y
                # (the complex transposed product is far slower on the device)
                cre = Vr @ torch.view_as_real(w).reshape(2 * n)
                cim = Vr @ torch.view_as_real(-1j * w).reshape(2 * n)
                c = torch.complex(cre, cim)
                w = w - c @ V[: j + 1]
                h += c
            beta = torch.linalg.vector_norm(w)
            H[: j + 1, j] = h.cpu().numpy()
            H[j + 1, j] = float(beta)
            V[j + 1] = w / beta
        Hm = H[:m, :m]
        theta, Y = np.linalg.eig(Hm)
        order = np.argsort(theta.real)
        resid = np.abs(H[m, m - 1]) * np.abs(Y[m - 1, order[:nev]]) / np.maximum(np.abs(theta[order[:nev]]), 1e-300)
        if log:
            log("mcrit: restart %d, %d matvecs, smallest Re theta %.8f, residuals %s" %
                (restart, matvecs, theta[order[0]].real, np.array2string(resid, precision=2)))
        out_of_time = max_seconds is not None and time.time() - t_start > max_seconds
        if np.all(resid <= tol) or restart == max_restarts or out_of_time:
            return theta[order[:nev]], resid, matvecs, restart
        # Schur form with the `keep` smallest-real-part Ritz values first
        thr = np.sort(theta.real)[keep - 1]
        T, Z, sdim = sla.schur(Hm, output="complex", sort=lambda x: x.real <= thr)
        kk = int(sdim)
        if kk < nev:
            kk = keep
        Zt = torch.as_tensor(Z[:, :kk].T.copy(), device=device)   # (kk, m)
        for c0 in range(0, n, chunk):
            c1 = min(n, c0 + chunk)
            V[:kk, c0:c1] = Zt @ V[:m, c0:c1]
        V[kk] = V[m]
        Hn = np.zeros_like(H)
        Hn[:kk, :kk] = T[:kk, :kk]
        Hn[kk, :kk] = H[m, m - 1] * Z[m - 1, :kk]
        H = Hn
        k = kk
    raise AssertionError("unreachable")


def m_crit(dims, gauge, csw=1.0, nev=2, m=64, tol=1e-4, log=None, **kw):
    """m_crit = -Re lambda_SR(D(m0 = 0)) with D applied by the library (FP64)."""
    import torch

    import paper_1303_1377_amd as G

    dims = tuple(int(v) for v in dims)
    vol = int(np.prod(dims))
    s = G.Solver(dims, gauge, 0.0, csw)
    # a minimal configuration gives dd_apply a resident staging buffer
    s.configure(G.default_params(levels=2, n_tv=[2], outer_restart=1, coarse_restart=1, mid_restart=1,
                                 max_rhs=1, precision=64))

    def apply(v):
        out, _ = s.apply("D", 0, v.view(vol, 4, 3))
        return out.reshape(-1)

    t0 = time.time()
    ev, res, mv, rs = smallest_real_eigs(apply, vol * 12, nev=nev, m=m, tol=tol, log=log, **kw)
    torch.cuda.synchronize()
    s.close()
    return dict(m_crit=float(-ev[0].real), eigenvalues=[[float(e.real), float(e.imag)] for e in ev],
                residuals=[float(r) for r in res], matvecs=int(mv), restarts=int(rs), seconds=time.time() - t0,
                method="Krylov-Schur (m=%d, keep=%d) on the library's FP64 D(m0=0), smallest real part, "
                       "relative Ritz residual target %.0e" % (m, kw.get("keep") or max(nev + 2, m // 2), tol))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", required=True)
    ap.add_argument("--eps", type=float, default=0.4)
    ap.add_argument("--ape", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--csw", type=float, default=1.0)
    ap.add_argument("--device-field", action="store_true", help="draw the links on the GPU (large lattices)")
    ap.add_argument("--m", type=int, default=64)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--max-seconds", type=float, default=None)
    a = ap.parse_args()
    from paper_1303_1377_amd import fields as F

    def log(*x):
        print(*x, file=sys.stderr, flush=True)

    dims = tuple(int(v) for v in a.dims.split(","))
    t = time.time()
    if a.device_field:
        U = F.make_gauge_device(dims, a.eps, a.seed, ape_steps=a.ape, ape_alpha=0.5)
    else:
        U = F.make_gauge(dims, a.eps, a.seed, ape_steps=a.ape, ape_alpha=0.5)
    log("mcrit: field %s in %.1fs" % (a.dims, time.time() - t))
    r = m_crit(dims, U, a.csw, m=a.m, tol=a.tol, log=log, max_seconds=a.max_seconds)
    r.update(dims=list(dims), eps=a.eps, ape=a.ape, seed=a.seed, csw=a.csw,
             field="device" if a.device_field else "host")
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
