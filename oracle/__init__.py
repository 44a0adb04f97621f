"""ctypes binding of the plain FP64 CPU oracle (oracle/ddamg_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product path never imports this package.

Array conventions follow the public layout of the solver: complex128, canonical
site order ((x0*N1+x1)*N2+x2)*N3+x3, fine spinors [site][spin][colour],
gauge [site][mu][3][3], coarse vectors [site][2N] with index h*N + k.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ddamg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAXLEV = 4


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("levels", C.c_int),
        ("n_tv", C.c_int * MAXLEV),
        ("agg", (C.c_int * 4) * MAXLEV),
        ("sap", (C.c_int * 4) * MAXLEV),
        ("mr_steps", C.c_int * MAXLEV),
        ("nu", C.c_int),
        ("n_inv", C.c_int),
        ("coarse_tol", C.c_double),
        ("coarse_restart", C.c_int),
        ("coarse_maxit", C.c_int),
        ("coarse_fixed", C.c_int),
        ("mid_tol", C.c_double),
        ("mid_restart", C.c_int),
        ("mid_maxit", C.c_int),
        ("mid_fixed", C.c_int),
        ("outer_restart", C.c_int),
        ("outer_maxit", C.c_int),
        ("id_setup", C.c_int),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("outer_iters", C.c_int),
        ("restarts", C.c_int),
        ("coarse_iters", C.c_long * MAXLEV),
        ("true_relres", C.c_double),
        ("converged", C.c_int),
    ]


# Default parameters: Table 1 of the paper (two levels).
DEFAULTS = dict(
    levels=2,
    n_tv=[20, 20, 20, 20],
    agg=[[4, 4, 4, 4], [2, 2, 2, 2], [2, 2, 2, 2], [2, 2, 2, 2]],
    sap=[[4, 4, 4, 4], [2, 2, 2, 2], [2, 2, 2, 2], [2, 2, 2, 2]],
    mr_steps=[4, 4, 4, 4],
    nu=2,
    n_inv=6,
    coarse_tol=5e-2,
    coarse_restart=30,
    coarse_maxit=1000,
    coarse_fixed=0,
    mid_tol=5e-2,
    mid_restart=10,
    mid_maxit=50,
    mid_fixed=0,
    outer_restart=25,
    outer_maxit=2000,
    id_setup=0,
)


def make_params(**kw) -> Params:
    d = dict(DEFAULTS)
    for k, v in kw.items():
        if k not in d:
            raise KeyError(k)
        d[k] = v
    p = Params()
    p.levels = d["levels"]
    for l in range(MAXLEV):
        p.n_tv[l] = d["n_tv"][l] if l < len(d["n_tv"]) else 0
        p.mr_steps[l] = d["mr_steps"][l] if l < len(d["mr_steps"]) else 4
        for mu in range(4):
            p.agg[l][mu] = d["agg"][l][mu] if l < len(d["agg"]) else 2
            p.sap[l][mu] = d["sap"][l][mu] if l < len(d["sap"]) else 2
    for k in ("nu", "n_inv", "coarse_restart", "coarse_maxit", "coarse_fixed",
              "mid_restart", "mid_maxit", "mid_fixed", "outer_restart", "outer_maxit", "id_setup"):
        setattr(p, k, int(d[k]))
    p.coarse_tol = float(d["coarse_tol"])
    p.mid_tol = float(d["mid_tol"])
    return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=False)
        L = C.CDLL(_LIB)
        vp, cp, ip, dp = C.c_void_p, C.c_void_p, C.POINTER(C.c_int), C.c_double
        L.or_create.restype = vp
        L.or_create.argtypes = [ip, cp, cp, dp, dp]
        L.or_destroy.argtypes = [vp]
        L.or_error.restype = C.c_char_p
        L.or_error.argtypes = [vp]
        L.or_gamma.argtypes = [cp]
        L.or_clover_offblock.restype = C.c_double
        L.or_clover_offblock.argtypes = [ip, cp, dp]
        L.or_clover_site.argtypes = [ip, cp, dp, C.c_long, cp]
        L.or_get_clover.argtypes = [vp, cp, cp]
        L.or_shift_mass.argtypes = [vp, dp]
        L.or_level_info.argtypes = [vp, C.c_int, ip, ip]
        L.or_apply.argtypes = [vp, C.c_int, cp, cp]
        L.or_configure.argtypes = [vp, C.POINTER(Params)]
        L.or_set_vectors.argtypes = [vp, C.c_int, cp]
        L.or_get_vectors.argtypes = [vp, C.c_int, cp]
        L.or_build.argtypes = [vp, C.c_int]
        L.or_get_P.argtypes = [vp, C.c_int, cp]
        L.or_set_P.argtypes = [vp, C.c_int, cp]
        L.or_get_coarse.argtypes = [vp, C.c_int, cp, cp]
        L.or_restrict.argtypes = [vp, C.c_int, cp, cp]
        L.or_prolong.argtypes = [vp, C.c_int, cp, cp]
        L.or_sap.argtypes = [vp, C.c_int, cp, cp, C.c_int, C.c_int]
        L.or_block_solve.argtypes = [vp, C.c_int, C.c_long, cp, cp]
        L.or_coarse_solve.restype = C.c_long
        L.or_coarse_solve.argtypes = [vp, C.c_int, cp, cp]
        L.or_schur.argtypes = [vp, C.c_int, cp, cp]
        L.or_vcycle.argtypes = [vp, C.c_int, C.c_int, cp, cp]
        L.or_bicgstab.restype = C.c_long
        L.or_bicgstab.argtypes = [vp, cp, cp, C.c_int]
        L.or_solve_bicgstab.argtypes = [vp, cp, cp, dp, C.c_int, C.POINTER(Stats)]
        L.or_solve_id.argtypes = [vp, cp, cp, dp, C.c_int, C.POINTER(Stats)]
        L.or_apply_deflated.argtypes = [vp, cp, cp]
        L.or_fgmres_level.restype = C.c_long
        L.or_fgmres_level.argtypes = [vp, C.c_int, cp, cp]
        L.or_setup_level.argtypes = [vp, C.c_int]
        L.or_setup.argtypes = [vp, C.POINTER(C.c_void_p)]
        L.or_solve.argtypes = [vp, cp, cp, dp, C.c_long, C.POINTER(Stats)]
        L.or_mark_setup.argtypes = [vp]
        L.or_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _c(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _dims(d):
    return (C.c_int * 4)(*[int(v) for v in d])


def gamma_matrices() -> np.ndarray:
    out = np.zeros((4, 4, 4), dtype=np.complex128)
    lib().or_gamma(_ptr(out))
    return out


def clover_site(dims, gauge, csw, site) -> np.ndarray:
    g = _c(gauge)
    out = np.zeros((12, 12), dtype=np.complex128)
    lib().or_clover_site(_dims(dims), _ptr(g), float(csw), int(site), _ptr(out))
    return out


def clover_offblock(dims, gauge, csw) -> float:
    g = _c(gauge)
    return lib().or_clover_offblock(_dims(dims), _ptr(g), float(csw))


def num_threads() -> int:
    return lib().or_num_threads()


class Oracle:
    """FP64 CPU DD-alpha-AMG on one gauge field."""

    def __init__(self, dims, gauge, m0, csw, clover_T=None):
        self.dims = tuple(int(v) for v in dims)
        self.vol = int(np.prod(self.dims))
        g = _c(gauge)
        assert g.size == self.vol * 36
        ct = None if clover_T is None else _c(clover_T)
        h = lib().or_create(_dims(self.dims), _ptr(g), None if ct is None else _ptr(ct), float(m0), float(csw))
        if not h:
            raise ValueError("oracle: invalid lattice dims %r" % (self.dims,))
        self.h = h
        self.m0, self.csw = m0, csw
        self.params = None

    def close(self):
        if getattr(self, "h", None):
            lib().or_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # ---- geometry --------------------------------------------------------
    def level_info(self, l):
        d = (C.c_int * 4)()
        nd = C.c_int()
        if lib().or_level_info(self.h, l, d, C.byref(nd)):
            raise ValueError("no level %d" % l)
        return tuple(d), nd.value

    def level_size(self, l):
        d, nd = self.level_info(l)
        return int(np.prod(d)), nd

    # ---- operator --------------------------------------------------------
    def apply(self, psi, level=0):
        vol, nd = self.level_size(level)
        x = _c(psi).reshape(vol * nd)
        out = np.empty_like(x)
        lib().or_apply(self.h, level, _ptr(x), _ptr(out))
        return out.reshape(np.shape(psi))

    def clover(self):
        A = np.zeros((self.vol, 2, 6, 6), dtype=np.complex128)
        Ai = np.zeros_like(A)
        lib().or_get_clover(self.h, _ptr(A), _ptr(Ai))
        return A, Ai

    def shift_mass(self, dm):
        lib().or_shift_mass(self.h, float(dm))

    # ---- multigrid components -------------------------------------------
    def configure(self, **kw):
        self.params = make_params(**kw)
        if lib().or_configure(self.h, C.byref(self.params)):
            raise ValueError("oracle configure: " + lib().or_error(self.h).decode())

    def set_vectors(self, l, v):
        vol, nd = self.level_size(l)
        a = _c(v)
        assert a.size == self.params.n_tv[l] * vol * nd
        lib().or_set_vectors(self.h, l, _ptr(a))

    def get_vectors(self, l):
        vol, nd = self.level_size(l)
        out = np.zeros((self.params.n_tv[l], vol, nd), dtype=np.complex128)
        lib().or_get_vectors(self.h, l, _ptr(out))
        return out

    def build(self, l):
        if lib().or_build(self.h, l):
            raise RuntimeError("oracle build: " + lib().or_error(self.h).decode())

    def get_P(self, l):
        vol, nd = self.level_size(l)
        out = np.zeros((self.params.n_tv[l], vol, nd), dtype=np.complex128)
        lib().or_get_P(self.h, l, _ptr(out))
        return out

    def set_P(self, l, P):
        a = _c(P)
        if lib().or_set_P(self.h, l, _ptr(a)):
            raise RuntimeError("oracle set_P failed")

    def get_coarse(self, l):
        vol, nd = self.level_size(l)
        M = np.zeros((vol, 9, nd, nd), dtype=np.complex128)
        Mi = np.zeros((vol, nd, nd), dtype=np.complex128)
        lib().or_get_coarse(self.h, l, _ptr(M), _ptr(Mi))
        return M, Mi

    def restrict(self, l, v):
        volc, ndc = self.level_size(l + 1)
        a = _c(v)
        out = np.zeros(volc * ndc, dtype=np.complex128)
        lib().or_restrict(self.h, l, _ptr(a), _ptr(out))
        return out.reshape(volc, ndc)

    def prolong(self, l, vc):
        vol, nd = self.level_size(l)
        a = _c(vc)
        out = np.zeros(vol * nd, dtype=np.complex128)
        lib().or_prolong(self.h, l, _ptr(a), _ptr(out))
        return out.reshape(vol, nd)

    def sap(self, l, rhs, nsweeps, z0=None):
        vol, nd = self.level_size(l)
        r = _c(rhs).reshape(vol * nd)
        z = np.zeros(vol * nd, dtype=np.complex128) if z0 is None else _c(z0).reshape(vol * nd).copy()
        lib().or_sap(self.h, l, _ptr(r), _ptr(z), int(nsweeps), 1 if z0 is None else 0)
        return z.reshape(np.shape(rhs))

    def block_solve(self, l, block, r, z0=None):
        vol, nd = self.level_size(l)
        rr = _c(r).reshape(vol * nd)
        z = np.zeros(vol * nd, dtype=np.complex128) if z0 is None else _c(z0).reshape(vol * nd).copy()
        lib().or_block_solve(self.h, l, int(block), _ptr(rr), _ptr(z))
        return z.reshape(np.shape(r))

    def coarse_solve(self, l, r):
        vol, nd = self.level_size(l)
        rr = _c(r).reshape(vol * nd)
        e = np.zeros_like(rr)
        its = lib().or_coarse_solve(self.h, l, _ptr(rr), _ptr(e))
        return e.reshape(np.shape(r)), its

    def schur(self, l, v):
        vol, nd = self.level_size(l)
        a = _c(v).reshape(vol * nd)
        out = np.zeros_like(a)
        lib().or_schur(self.h, l, _ptr(a), _ptr(out))
        return out.reshape(np.shape(v))

    def vcycle(self, l, r, bottom=None):
        if bottom is None:
            bottom = self.params.levels - 1
        vol, nd = self.level_size(l)
        rr = _c(r).reshape(vol * nd)
        z = np.zeros_like(rr)
        lib().or_vcycle(self.h, l, bottom, _ptr(rr), _ptr(z))
        return z.reshape(np.shape(r))

    def fgmres_level(self, l, r):
        """Intermediate-level FGMRES (3+ levels) on level l: (solution, iterations)."""
        vol, nd = self.level_size(l)
        rr = _c(r).reshape(vol * nd)
        x = np.zeros_like(rr)
        its = lib().or_fgmres_level(self.h, l, _ptr(rr), _ptr(x))
        return x.reshape(np.shape(r)), its

    def setup_level(self, l):
        if lib().or_setup_level(self.h, l):
            raise RuntimeError("oracle setup: " + lib().or_error(self.h).decode())

    def setup(self, tvs):
        arrs = [_c(v) for v in tvs]
        ptrs = (C.c_void_p * MAXLEV)(*([a.ctypes.data for a in arrs] + [None] * (MAXLEV - len(arrs))))
        if lib().or_setup(self.h, ptrs):
            raise RuntimeError("oracle setup: " + lib().or_error(self.h).decode())

    def bicgstab(self, b, steps):
        """Odd-even BiCGStab (steps from zero) + back-substitution: ~D^{-1} b."""
        bb = _c(b).reshape(self.vol * 12)
        x = np.zeros_like(bb)
        its = lib().or_bicgstab(self.h, _ptr(bb), _ptr(x), int(steps))
        return x.reshape(np.shape(b)), its

    def solve_bicgstab(self, b, tol=1e-10, steps=50):
        """FGMRES(outer_restart) preconditioned by `steps` odd-even BiCGStab steps."""
        bb = _c(b).reshape(self.vol * 12)
        x = np.zeros_like(bb)
        st = Stats()
        rc = lib().or_solve_bicgstab(self.h, _ptr(bb), _ptr(x), float(tol), int(steps), C.byref(st))
        return x.reshape(np.shape(b)), dict(rc=rc, outer_iters=st.outer_iters, restarts=st.restarts,
                                            true_relres=st.true_relres, converged=bool(st.converged))

    def solve_id(self, b, tol=1e-10, nu=5):
        """Inexact deflation (two-level hierarchy as built): FGMRES on D pi_R with
        nu SAP iterations as preconditioner; returns (x, stats)."""
        bb = _c(b).reshape(self.vol * 12)
        x = np.zeros_like(bb)
        st = Stats()
        rc = lib().or_solve_id(self.h, _ptr(bb), _ptr(x), float(tol), int(nu), C.byref(st))
        return x.reshape(np.shape(b)), dict(rc=rc, outer_iters=st.outer_iters, restarts=st.restarts,
                                            coarse_iters=list(st.coarse_iters), true_relres=st.true_relres,
                                            converged=bool(st.converged))

    def apply_deflated(self, v):
        """D pi_R v (inexact-deflation operator; coarse solves to the parameters' tolerance)."""
        a = _c(v).reshape(self.vol * 12)
        out = np.zeros_like(a)
        lib().or_apply_deflated(self.h, _ptr(a), _ptr(out))
        return out.reshape(np.shape(v))

    def mark_setup(self):
        lib().or_mark_setup(self.h)

    def solve(self, b, tol=1e-10, fixed=0):
        bb = _c(b).reshape(self.vol * 12)
        x = np.zeros_like(bb)
        st = Stats()
        rc = lib().or_solve(self.h, _ptr(bb), _ptr(x), float(tol), int(fixed), C.byref(st))
        stats = dict(
            rc=rc,
            outer_iters=st.outer_iters,
            restarts=st.restarts,
            coarse_iters=list(st.coarse_iters),
            true_relres=st.true_relres,
            converged=bool(st.converged),
        )
        return x.reshape(np.shape(b)), stats
