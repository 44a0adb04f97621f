"""MI355X DD-alpha-AMG solver for the clover-improved Wilson Dirac system.

Thin ctypes binding of libddamg.so (C-ABI in include/ddamg.h): argument
marshalling only; every step of the method runs in the HIP kernels of the
library.  PyTorch provides device memory (complex128 tensors on the HIP device)
and the stream.  Importing the package never loads the library; the first use
of a solver does, and raises if the library was not built.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

__all__ = ["Solver", "Params", "Stats", "default_params", "library", "DDError", "OPS", "KERNEL_CLASSES"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddamg.so")
MAXLEV = 4

KERNEL_CLASSES = ["dirac64", "dirac_prec", "sap", "restrict", "prolong", "coarse", "coarse_sap", "reduce", "blas",
                  "coarse_step"]
OPS = dict(D=0, D_PREC=1, SAP=2, VCYCLE=3, RESTRICT=4, PROLONG=5, COARSE_SOLVE=6, SCHUR=7, FGMRES=8, BICGSTAB=9,
           DEFLATED=10)
# DD_SCHED_* flags of include/ddamg.h
SCHED = dict(FUSED=1, XCD=2, LDS=4, NO_MFMA=8, GRAPH=16, COOP=32, COOP_ABORT=64)
STATUS = {0: "DD_OK", -1: "DD_EINVAL", -2: "DD_ENOMEM", -3: "DD_ENOCONV", -4: "DD_EDEVICE", -5: "DD_ESTATE",
          -6: "DD_ENUMERIC"}


class DDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


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
        ("precision", C.c_int),
        ("given_vectors", C.c_int),
        ("seed", C.c_ulonglong),
        ("max_rhs", C.c_int),
        ("id_setup", C.c_int),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("outer_iters", C.c_int),
        ("restarts", C.c_int),
        ("coarse_iters", C.c_long * MAXLEV),
        ("true_relres", C.c_double),
        ("setup_s", C.c_double),
        ("solve_s", C.c_double),
        ("converged", C.c_int),
    ]

    def as_dict(self):
        return dict(outer_iters=self.outer_iters, restarts=self.restarts, coarse_iters=list(self.coarse_iters),
                    true_relres=self.true_relres, setup_s=self.setup_s, solve_s=self.solve_s,
                    converged=bool(self.converged))


_lib = None


def library():
    """Load libddamg.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libddamg.so not built: run paper_1303_1377_amd/build.py (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, ip, dp = C.c_void_p, C.POINTER(C.c_int), C.c_double
        L.dd_default_params.argtypes = [C.POINTER(Params)]
        L.dd_last_error.restype = C.c_char_p
        L.dd_last_error.argtypes = [vp]
        L.dd_create.argtypes = [C.POINTER(vp), ip, vp, vp, dp, dp, vp]
        L.dd_destroy.argtypes = [vp]
        L.dd_setup.argtypes = [vp, C.c_int, ip, C.c_int, C.POINTER(Params)]
        L.dd_solve.argtypes = [vp, vp, vp, dp, C.POINTER(Stats)]
        L.dd_solve_batch.argtypes = [vp, C.c_int, vp, vp, dp, C.POINTER(Stats)]
        L.dd_set_mass.argtypes = [vp, dp]
        L.dd_configure.argtypes = [vp, C.POINTER(Params)]
        L.dd_set_test_vectors.argtypes = [vp, C.c_int, C.c_int, vp]
        L.dd_get_test_vectors.argtypes = [vp, C.c_int, vp]
        L.dd_build_level.argtypes = [vp, C.c_int]
        L.dd_mark_setup.argtypes = [vp]
        L.dd_get_P.argtypes = [vp, C.c_int, vp]
        L.dd_get_coarse.argtypes = [vp, C.c_int, vp, vp]
        L.dd_get_clover.argtypes = [vp, vp, vp]
        L.dd_apply.argtypes = [vp, C.c_int, C.c_int, C.c_int, vp, vp, C.POINTER(C.c_long)]
        L.dd_apply_batch.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, vp, vp, C.POINTER(C.c_long)]
        L.dd_apply_D_noalloc.argtypes = [vp, vp, vp]
        L.dd_solve_bicgstab.argtypes = [vp, vp, vp, dp, C.c_int, C.c_int, C.POINTER(Stats)]
        L.dd_solve_id.argtypes = [vp, vp, vp, dp, C.c_int, dp, C.POINTER(Stats)]
        L.dd_stream_load.argtypes = [vp, C.c_int, vp, dp]
        L.dd_stream_cycle.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(Stats)]
        L.dd_stream_take.argtypes = [vp, C.c_int, vp, C.POINTER(Stats)]
        L.dd_level_info.argtypes = [vp, C.c_int, ip, ip]
        L.dd_profile.argtypes = [vp, C.c_int]
        L.dd_profile_classes.argtypes = [vp, C.c_uint]
        L.dd_profile_read.argtypes = [vp, C.c_int, C.POINTER(C.c_long), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.dd_time_kernel.argtypes = [vp, C.c_int, C.c_int, C.POINTER(C.c_double)]
        L.dd_device_bytes.restype = C.c_longlong
        L.dd_device_bytes.argtypes = [vp]
        L.dd_set_schedule.argtypes = [vp, C.c_int]
        L.dd_get_schedule.argtypes = [vp]
        L.dd_get_schedule.restype = C.c_int
        L.dd_autotune.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.dd_autotune_coarse.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.dd_autotune_cached.argtypes = [vp, C.c_char_p, C.c_int, ip, ip, ip]
        for name in ("dd_create", "dd_setup", "dd_solve", "dd_solve_batch", "dd_set_mass", "dd_configure",
                     "dd_set_test_vectors", "dd_get_test_vectors", "dd_build_level", "dd_mark_setup", "dd_get_P",
                     "dd_get_coarse", "dd_get_clover", "dd_apply", "dd_level_info", "dd_profile", "dd_profile_read",
                     "dd_profile_classes", "dd_apply_D_noalloc", "dd_stream_load", "dd_stream_cycle", "dd_stream_take",
                     "dd_solve_bicgstab", "dd_solve_id", "dd_autotune_cached",
                     "dd_time_kernel", "dd_set_schedule", "dd_autotune", "dd_apply_batch", "dd_autotune_coarse"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def default_params(**kw) -> Params:
    """Table 1 defaults, overridden by keyword (lists for per-level fields)."""
    p = Params()
    library().dd_default_params(C.byref(p))
    for k, v in kw.items():
        if k in ("n_tv", "mr_steps"):
            for l, x in enumerate(v):
                getattr(p, k)[l] = int(x)
        elif k in ("agg", "sap"):
            for l, blk in enumerate(v):
                for mu in range(4):
                    getattr(p, k)[l][mu] = int(blk[mu])
        elif k in ("coarse_tol", "mid_tol"):
            setattr(p, k, float(v))
        elif k == "seed":
            p.seed = int(v)
        else:
            setattr(p, k, int(v))
    return p


def _torch():
    import torch

    return torch


def _dev(t):
    """Device complex128 contiguous tensor for an array-like."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    return t.to(device="cuda", dtype=torch.complex128).contiguous()


_live = weakref.WeakSet()


@atexit.register
def _close_live_solvers():
    """Release every context still open when the interpreter exits, while the
    HIP runtime (and any profiler attached to it) is still fully alive; left
    to garbage collection the contexts would be destroyed during the runtime's
    own teardown."""
    for s in list(_live):
        try:
            s.close()
        except Exception:
            pass


def _order_after_current(stream):
    """Make `stream` wait for the work torch queued on its current stream (the
    conversions and copies that produced the input tensors), so the library,
    which enqueues on `stream`, reads them only after they are written."""
    torch = _torch()
    cur = torch.cuda.current_stream()
    if stream is not None and stream != cur:
        stream.wait_stream(cur)


class Solver:
    """One gauge field, one hierarchy (see include/ddamg.h for the semantics).

    Inputs are prepared on torch's current stream and the library runs on
    `self.stream`; every call that reads caller data first orders the solver's
    stream after the current one.  Calls return after their work has finished
    (the C-ABI synchronises its stream), so outputs are ready on return."""

    def __init__(self, dims, gauge, m0, csw, clover=None, stream=None):
        torch = _torch()
        L = library()
        self.dims = tuple(int(v) for v in dims)
        self.vol = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]
        g = _dev(gauge).reshape(self.vol, 4, 3, 3)
        cl = None if clover is None else _dev(clover).reshape(self.vol, 2, 6, 6)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        _order_after_current(self.stream)
        h = C.c_void_p()
        rc = L.dd_create(C.byref(h), (C.c_int * 4)(*self.dims), C.c_void_p(g.data_ptr()),
                         None if cl is None else C.c_void_p(cl.data_ptr()), float(m0), float(csw),
                         C.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise DDError(rc, L.dd_last_error(None).decode())
        self.h = h
        self.m0, self.csw = float(m0), float(csw)
        self.params = None
        _live.add(self)

    # ---- plumbing ----------------------------------------------------------
    def _check(self, rc, ok=(0,)):
        if rc not in ok:
            raise DDError(rc, library().dd_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            library().dd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_info(self, level):
        d = (C.c_int * 4)()
        nd = C.c_int()
        self._check(library().dd_level_info(self.h, level, d, C.byref(nd)))
        return tuple(d), nd.value

    def level_size(self, level):
        d, nd = self.level_info(level)
        return d[0] * d[1] * d[2] * d[3], nd

    def device_bytes(self):
        return int(library().dd_device_bytes(self.h))

    # ---- main API ----------------------------------------------------------
    def setup(self, n_tv=0, block=None, levels=0, params=None, **kw):
        p = params if params is not None else default_params(**kw)
        blk = None if block is None else (C.c_int * 4)(*block)
        self._check(library().dd_setup(self.h, int(n_tv), blk, int(levels), C.byref(p)))
        self.params = p

    def configure(self, params=None, **kw):
        p = params if params is not None else default_params(**kw)
        self._check(library().dd_configure(self.h, C.byref(p)))
        self.params = p

    def solve(self, b, tol=1e-10, allow_noconv=False):
        torch = _torch()
        bb = _dev(b).reshape(self.vol, 4, 3)
        x = torch.empty_like(bb)
        st = Stats()
        _order_after_current(self.stream)
        rc = library().dd_solve(self.h, C.c_void_p(bb.data_ptr()), C.c_void_p(x.data_ptr()), float(tol), C.byref(st))
        self._check(rc, ok=(0, -3) if allow_noconv else (0,))
        return x, st.as_dict()

    def solve_batch(self, b, tol=1e-10, allow_noconv=False):
        """k right-hand sides [k][vol][4][3] in batches of at most max_rhs."""
        torch = _torch()
        bb = _dev(b).reshape(-1, self.vol, 4, 3).contiguous()
        k = bb.shape[0]
        x = torch.empty_like(bb)
        st = (Stats * max(k, 1))()
        _order_after_current(self.stream)
        rc = library().dd_solve_batch(self.h, k, C.c_void_p(bb.data_ptr()), C.c_void_p(x.data_ptr()), float(tol), st)
        self._check(rc, ok=(0, -3) if allow_noconv else (0,))
        return x, [s.as_dict() for s in st[:k]]

    # ---- continuous batching ---------------------------------------------------
    SLOT_FREE, SLOT_RUNNING, SLOT_CONVERGED, SLOT_STOPPED = 0, 1, 2, 3

    def stream_load(self, slot, b, tol=1e-10):
        """Put one right-hand side [vol][4][3] into a free slot of the outer FGMRES."""
        bb = _dev(b).reshape(self.vol, 4, 3)
        _order_after_current(self.stream)
        self._check(library().dd_stream_load(self.h, int(slot), C.c_void_p(bb.data_ptr()), float(tol)))

    def stream_cycle(self):
        """One restart cycle of every running slot; returns ([slot states], [stats dicts])."""
        R = int(self.params.max_rhs)
        state = (C.c_int * R)()
        st = (Stats * R)()
        self._check(library().dd_stream_cycle(self.h, state, st))
        return list(state), [s.as_dict() for s in st]

    def stream_take(self, slot, allow_noconv=False):
        """Solution and stats of a finished slot; frees the slot."""
        torch = _torch()
        x = torch.empty((self.vol, 4, 3), dtype=torch.complex128, device="cuda")
        st = Stats()
        rc = library().dd_stream_take(self.h, int(slot), C.c_void_p(x.data_ptr()), C.byref(st))
        self._check(rc, ok=(0, -3) if allow_noconv else (0,))
        return x, st.as_dict()

    def solve_bicgstab(self, b, tol=1e-10, steps=50, precision=32, allow_noconv=False):
        """The comparison solver: FP64 FGMRES preconditioned by `steps` odd-even
        BiCGStab steps in `precision` (needs configure())."""
        torch = _torch()
        bb = _dev(b).reshape(self.vol, 4, 3)
        x = torch.empty_like(bb)
        st = Stats()
        _order_after_current(self.stream)
        rc = library().dd_solve_bicgstab(self.h, C.c_void_p(bb.data_ptr()), C.c_void_p(x.data_ptr()), float(tol),
                                         int(steps), int(precision), C.byref(st))
        self._check(rc, ok=(0, -3) if allow_noconv else (0,))
        return x, st.as_dict()

    def solve_id(self, b, tol=1e-10, nu=5, coarse_tol=1e-12, allow_noconv=False):
        """The second comparison solver, inexact deflation (FP64, two-level
        setup): FGMRES on D pi_R preconditioned by nu SAP iterations, coarse
        systems solved to coarse_tol."""
        torch = _torch()
        bb = _dev(b).reshape(self.vol, 4, 3)
        x = torch.empty_like(bb)
        st = Stats()
        _order_after_current(self.stream)
        rc = library().dd_solve_id(self.h, C.c_void_p(bb.data_ptr()), C.c_void_p(x.data_ptr()), float(tol), int(nu),
                                   float(coarse_tol), C.byref(st))
        self._check(rc, ok=(0, -3) if allow_noconv else (0,))
        return x, st.as_dict()

    def set_mass(self, m0):
        self._check(library().dd_set_mass(self.h, float(m0)))
        self.m0 = float(m0)

    # ---- live kernel timing --------------------------------------------------
    def profile(self, enable=True, classes=None):
        """Start (reset) or stop live timing; `classes` limits it to the named
        kernel classes (the others run without events)."""
        if classes is None or not enable:
            self._check(library().dd_profile(self.h, 1 if enable else 0))
        else:
            mask = 0
            for name in classes:
                mask |= 1 << KERNEL_CLASSES.index(name)
            self._check(library().dd_profile_classes(self.h, mask))

    def profile_read(self):
        """{class: (launches, total_ms, algorithmic_bytes)} since profile(True)."""
        out = {}
        for k, name in enumerate(KERNEL_CLASSES):
            n, ms, by = C.c_long(), C.c_double(), C.c_double()
            self._check(library().dd_profile_read(self.h, k, C.byref(n), C.byref(ms), C.byref(by)))
            out[name] = (n.value, ms.value, by.value)
        return out

    # ---- launch schedules / autotuner -------------------------------------------
    def set_schedule(self, sched):
        self._check(library().dd_set_schedule(self.h, int(sched)))

    def get_schedule(self):
        return int(library().dd_get_schedule(self.h))

    def autotune(self, reps=10):
        """Time every fine-kernel schedule, keep the fastest; returns (chosen, [ms per schedule])."""
        ch = C.c_int()
        t = (C.c_double * 8)()
        self._check(library().dd_autotune(self.h, int(reps), C.byref(ch), t))
        return ch.value, list(t)

    def autotune_coarse(self, reps=3):
        """Step-by-step (single launches, graph replay) vs cooperative coarse GMRES (16..128
        workgroups), then single launches vs graph replay by whole solves; returns
        (grid or 0, [ms x 8])."""
        ch = C.c_int()
        t = (C.c_double * 8)()
        self._check(library().dd_autotune_coarse(self.h, int(reps), C.byref(ch), t))
        return ch.value, list(t)

    def autotune_cached(self, path=None, reps=3):
        """Apply the launch forms stored for this problem shape in the text cache
        at `path` (default: $DD_TUNE_CACHE, else ~/.cache/ddamg/autotune.txt), or
        tune them (autotune, then autotune_coarse) and store them; returns
        (schedule, cooperative grid, hit)."""
        if path is None:
            path = os.environ.get("DD_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "ddamg",
                                                                   "autotune.txt")
        d = os.path.dirname(os.path.abspath(path))
        os.makedirs(d, exist_ok=True)
        sc, gr, hit = C.c_int(), C.c_int(), C.c_int()
        self._check(library().dd_autotune_cached(self.h, os.fsencode(path), int(reps), C.byref(sc), C.byref(gr),
                                                 C.byref(hit)))
        return sc.value, gr.value, bool(hit.value)

    def time_kernel(self, name, reps=20):
        """Mean duration (ms) of one standalone launch: dirac64, dirac_prec or sap (full sweep)."""
        ms = C.c_double()
        self._check(library().dd_time_kernel(self.h, KERNEL_CLASSES.index(name), int(reps), C.byref(ms)))
        return ms.value

    # ---- components ----------------------------------------------------------
    def set_test_vectors(self, level, v):
        vv = _dev(v)
        n = int(vv.shape[0])
        _order_after_current(self.stream)
        self._check(library().dd_set_test_vectors(self.h, level, n, C.c_void_p(vv.data_ptr())))

    def get_test_vectors(self, level):
        torch = _torch()
        vol, nd = self.level_size(level)
        out = torch.empty((self.params.n_tv[level], vol, nd), dtype=torch.complex128, device="cuda")
        self._check(library().dd_get_test_vectors(self.h, level, C.c_void_p(out.data_ptr())))
        return out

    def build_level(self, level):
        self._check(library().dd_build_level(self.h, level))

    def mark_setup(self):
        self._check(library().dd_mark_setup(self.h))

    def get_P(self, level):
        torch = _torch()
        vol, nd = self.level_size(level)
        out = torch.empty((self.params.n_tv[level], vol, nd), dtype=torch.complex128, device="cuda")
        self._check(library().dd_get_P(self.h, level, C.c_void_p(out.data_ptr())))
        return out

    def get_coarse(self, level):
        torch = _torch()
        vol, nd = self.level_size(level)
        M = torch.empty((vol, 9, nd, nd), dtype=torch.complex128, device="cuda")
        Mi = torch.empty((vol, nd, nd), dtype=torch.complex128, device="cuda")
        self._check(library().dd_get_coarse(self.h, level, C.c_void_p(M.data_ptr()), C.c_void_p(Mi.data_ptr())))
        return M, Mi

    def get_clover(self):
        torch = _torch()
        A = torch.empty((self.vol, 2, 6, 6), dtype=torch.complex128, device="cuda")
        Ai = torch.empty_like(A)
        self._check(library().dd_get_clover(self.h, C.c_void_p(A.data_ptr()), C.c_void_p(Ai.data_ptr())))
        return A, Ai

    def apply(self, op, level, v, arg=0):
        """One component on device vectors (op: name in OPS or its code)."""
        torch = _torch()
        code = OPS[op] if isinstance(op, str) else int(op)
        vin = _dev(v)
        if code == OPS["RESTRICT"]:
            vol, nd = self.level_size(level + 1)
            out = torch.empty((vol, nd), dtype=torch.complex128, device="cuda")
        elif code == OPS["PROLONG"]:
            vol, nd = self.level_size(level)
            out = torch.empty((vol, nd), dtype=torch.complex128, device="cuda")
        else:
            out = torch.empty_like(vin)
        its = C.c_long(0)
        _order_after_current(self.stream)
        self._check(library().dd_apply(self.h, code, level, int(arg), C.c_void_p(vin.data_ptr()),
                                       C.c_void_p(out.data_ptr()), C.byref(its)))
        return out, its.value

    def apply_D_noalloc(self, v, out=None):
        """out = D v (fine level, FP64) through the allocation-free entry point;
        `out` may be a preallocated complex128 device tensor of v's shape."""
        torch = _torch()
        vin = _dev(v)
        if out is None:
            out = torch.empty_like(vin)
        _order_after_current(self.stream)
        self._check(library().dd_apply_D_noalloc(self.h, C.c_void_p(vin.data_ptr()), C.c_void_p(out.data_ptr())))
        return out

    def apply_batch(self, op, level, vs, arg=0):
        """One component on k vectors at once ([k][vol_level][nd_level]); returns (out, [iters])."""
        torch = _torch()
        code = OPS[op] if isinstance(op, str) else int(op)
        vin = _dev(vs)
        k = vin.shape[0]
        vin = vin.reshape(k, -1).contiguous()
        if code == OPS["RESTRICT"]:
            vol, nd = self.level_size(level + 1)
            out = torch.empty((k, vol, nd), dtype=torch.complex128, device="cuda")
        elif code == OPS["PROLONG"]:
            vol, nd = self.level_size(level)
            out = torch.empty((k, vol, nd), dtype=torch.complex128, device="cuda")
        else:
            vol, nd = self.level_size(level)
            out = torch.empty((k, vol, nd), dtype=torch.complex128, device="cuda")
        its = (C.c_long * k)()
        _order_after_current(self.stream)
        self._check(library().dd_apply_batch(self.h, code, level, int(arg), int(k), C.c_void_p(vin.data_ptr()),
                                             C.c_void_p(out.data_ptr()), its))
        return out, list(its)
