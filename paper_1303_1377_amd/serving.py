"""Continuous-batching solve server over the C-ABI.

Requests (a gauge field id, k right-hand sides, a tolerance) arrive at any
time.  The server

  * keeps the setup of each field (P, D_c, clover inverses: one solver
    context) resident on the device, admitted against an HBM budget and
    evicted least-recently-used when a new field needs room and the old one
    is idle;
  * batches right-hand sides that share a field: with a backend that offers
    continuous batching (dd_stream_*: the default solver) every slot of the
    outer FGMRES that finishes is refilled with the next queued RHS of the
    field between two restart cycles, while the other slots keep running; a
    backend with only solve_batch runs whole batches of one tolerance, RHS of
    different requests joining as batches start;
  * runs the batches of different fields concurrently, each field's context
    on its own HIP stream driven by its own worker thread, so their kernels
    overlap on the device;
  * records per-request latency (submit to last RHS done) and reports
    p50 / p99 latency and solves/s.

Every right-hand side's result is the one a single solve on the same resident
setup computes (the batched solver advances each RHS exactly as a single solve
would), so a request gives the same answer alone and in any mix.

The solver backend is injectable (`solver_factory`) so that the scheduling
logic can be exercised without a device.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field


@dataclass
class FieldSpec:
    """A registered gauge field: D(U, m0, csw) on a lattice `dims`."""

    dims: tuple
    gauge: object
    m0: float
    csw: float
    params: object = None       # Params for the setup (None: library defaults)
    clover: object = None
    est_bytes: int = 0          # HBM the resident setup is admitted with


@dataclass(eq=False)   # requests compare by identity (queue removal)
class _Request:
    field_id: object
    rhs: object                 # [k][vol][4][3] array-like
    tol: float
    future: Future
    t_submit: float
    k: int
    m0: float = None            # mass of this request (None: the field's own)
    next_rhs: int = 0           # first RHS not yet handed to a batch
    done: int = 0
    x: list = field(default_factory=list)
    stats: list = field(default_factory=list)


def _stack(xs):
    """Stack device tensors with torch and anything else with numpy."""
    try:
        import torch

        if isinstance(xs[0], torch.Tensor):
            return torch.stack([torch.as_tensor(x) for x in xs])
    except ImportError:  # pragma: no cover - torch is part of the image
        pass
    import numpy as np

    return np.stack([np.asarray(x) for x in xs])


def estimate_bytes(dims, params=None, max_rhs=1):
    """Device bytes a resident setup holds, following the library's
    allocations: fine fields (FP64 and FP32 copies), the outer FGMRES
    workspace for max_rhs right-hand sides, and per level the vector sets,
    test vectors, P, D_c, its self-block inverses (and on the coarsest level
    the folded even-site blocks) and the Krylov bases (FP16 copies for
    precision 16)."""
    def get(name, default):
        return getattr(params, name, default) if params is not None else default

    vol = 1
    for d in dims:
        vol *= d
    levels = get("levels", 2)
    prec = get("precision", 64)
    n_tv = list(get("n_tv", [20, 20, 20, 20]))
    agg = [tuple(a) for a in get("agg", [(4, 4, 4, 4)] + [(2, 2, 2, 2)] * 3)]
    m_out = get("outer_restart", 25)
    m_c = get("coarse_restart", 30)
    m_mid = get("mid_restart", 10)
    R = max_rhs
    sz = 16 if prec == 64 else 8            # complex entry of the preconditioner
    zb = 16 if prec == 64 else 8
    b = vol * 3168 + (9 << 20)              # links, clover, inverses (FP64 + FP32), canonical gauge
    nR = 12 * vol * R
    b += (m_out + 1) * nR * 16 + m_out * nR * zb + 4 * nR * 16
    if prec == 16:
        b += vol * 432                      # FP16 links and clover blocks
    n0 = 12 * vol
    b += 3 * R * n0 * sz + 2 * n_tv[0] * n0 * sz + (n_tv[0] * n0 * 4 if prec == 16 else 0)
    v = vol
    for l in range(1, levels):
        a = agg[l - 1]
        v //= a[0] * a[1] * a[2] * a[3]
        nd = 2 * n_tv[l - 1]
        nl = v * nd
        b += v * 10 * nd * nd * sz + (v * 10 * nd * nd * 4 if prec == 16 else 0)
        if l == levels - 1 and nd <= 64:   # even-site hop blocks with the self inverse folded in
            b += (v // 2) * 8 * nd * nd * (sz + (4 if prec == 16 else 0))
        b += 5 * R * nl * sz + R * 17 * 1024
        if l < levels - 1:
            b += 2 * n_tv[l] * nl * sz + (n_tv[l] * nl * 4 if prec == 16 else 0)
            b += (max(m_mid, m_c) + 1) * R * nl * sz + m_mid * R * nl * sz
        else:
            b += (m_c + 1) * R * nl * sz
    return int(b * 1.02) + (32 << 20)


class Server:
    """See the module docstring.  `submit` returns a Future resolving to
    (x [k][vol][4][3], [stats per RHS]); x is a device tensor, or a host
    tensor with results_on_host.  Right-hand sides may be host arrays: they
    stay on the host while queued and are copied to the device per batch, so
    queued requests hold no device memory."""

    def __init__(self, budget_bytes=200e9, max_rhs=12, solver_factory=None, clock=time.perf_counter,
                 results_on_host=False):
        self.budget = int(budget_bytes)
        self.results_on_host = bool(results_on_host)
        self.max_rhs = int(max_rhs)
        self.clock = clock
        self._factory = solver_factory or self._default_factory
        self._fields = {}
        self._resident = collections.OrderedDict()   # field_id -> solver (LRU order)
        self._resident_bytes = {}
        self._reserved = {}    # field_id -> bytes held for a setup that is being built
        self._busy = set()
        self._pending = collections.deque()
        self._cv = threading.Condition()
        self._closed = False
        self._latency = []
        self._solved = 0
        self._t_first = None
        self._t_last = None
        self.admitted = 0
        self.evicted = 0
        self._workers = {}
        self._dispatcher = threading.Thread(target=self._dispatch, name="dd-dispatch", daemon=True)
        self._dispatcher.start()

    # ---- registration / submission ------------------------------------------
    def add_field(self, field_id, dims, gauge, m0, csw, params=None, clover=None):
        spec = FieldSpec(tuple(dims), gauge, float(m0), float(csw), params, clover)
        spec.est_bytes = estimate_bytes(spec.dims, params, self.max_rhs)
        if spec.est_bytes > self.budget:
            raise ValueError("field %r needs about %.1f GB, above the HBM budget" % (field_id, spec.est_bytes / 1e9))
        with self._cv:
            self._fields[field_id] = spec

    def submit(self, field_id, b, tol=1e-10, m0=None):
        """Queue the solves of b (one RHS [vol][4][3] or k of them) on field
        `field_id`; with m0 the Dirac operator of that mass: the resident setup
        is moved to it (dd_set_mass: a diagonal shift, no new setup) for the
        batch, which only holds RHS of one mass."""
        import numpy as np

        if field_id not in self._fields:
            raise KeyError("unknown field %r" % (field_id,))
        spec = self._fields[field_id]
        vol = int(np.prod(spec.dims))
        shape = tuple(getattr(b, "shape", np.shape(b)))
        k = 1 if len(shape) == 3 else int(shape[0])
        rhs = b if len(shape) == 4 else b.reshape(1, vol, 4, 3)
        fut = Future()
        m = spec.m0 if m0 is None else float(m0)
        req = _Request(field_id, rhs, float(tol), fut, self.clock(), k, m0=m, x=[None] * k, stats=[None] * k)
        with self._cv:
            if self._closed:
                raise RuntimeError("server closed")
            if self._t_first is None:
                self._t_first = req.t_submit
            self._pending.append(req)
            self._cv.notify_all()
        return fut

    # ---- statistics -----------------------------------------------------------
    def stats(self):
        import numpy as np

        with self._cv:
            lat = np.array(self._latency) if self._latency else np.zeros(1)
            span = (self._t_last - self._t_first) if self._t_last and self._t_first else 0.0
            return dict(requests=len(self._latency), rhs_solved=self._solved,
                        p50_latency_s=float(np.percentile(lat, 50)), p99_latency_s=float(np.percentile(lat, 99)),
                        solves_per_s=(self._solved / span) if span > 0 else 0.0,
                        requests_per_s=(len(self._latency) / span) if span > 0 else 0.0,
                        resident=list(self._resident.keys()), resident_bytes=sum(self._resident_bytes.values()),
                        reserved_bytes=sum(self._reserved.values()),
                        admitted=self.admitted, evicted=self.evicted)

    def close(self):
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        self._dispatcher.join()
        for w in list(self._workers.values()):
            w.join()
        with self._cv:
            for fid in list(self._resident):
                self._evict(fid)

    # ---- internals ------------------------------------------------------------
    def _default_factory(self, spec):
        import torch

        import paper_1303_1377_amd as G

        stream = torch.cuda.Stream()
        s = G.Solver(spec.dims, spec.gauge, spec.m0, spec.csw, clover=spec.clover, stream=stream)
        p = spec.params if spec.params is not None else G.default_params()
        p.max_rhs = self.max_rhs
        s.setup(params=p)
        return s

    def _evict(self, fid):
        s = self._resident.pop(fid)
        self._resident_bytes.pop(fid, None)
        close = getattr(s, "close", None)
        if close:
            close()
        self.evicted += 1

    def _held(self):
        """Bytes of resident setups plus the reservations of setups being built."""
        return sum(self._resident_bytes.values()) + sum(self._reserved.values())

    def _admit(self, fid):
        """Make room for field `fid` (caller holds the lock).  True when the
        field may be set up now; its estimate is then reserved until the setup
        is resident (or has failed), so setups admitted together never exceed
        the budget."""
        need = self._fields[fid].est_bytes
        used = self._held()
        if used + need <= self.budget:
            self._reserved[fid] = need
            return True
        pending_fields = {r.field_id for r in self._pending}
        for old in list(self._resident):
            if used + need <= self.budget:
                break
            if old in self._busy or old in pending_fields:
                continue
            used -= self._resident_bytes.get(old, 0)
            self._evict(old)
        if used + need <= self.budget:
            self._reserved[fid] = need
            return True
        return False

    def _trim(self, keep):
        """Evict idle setups (least recently used first) while the resident
        bytes exceed the budget (caller holds the lock)."""
        pending_fields = {r.field_id for r in self._pending}
        for old in list(self._resident):
            if self._held() <= self.budget:
                break
            if old == keep or old in self._busy or old in pending_fields:
                continue
            self._evict(old)

    def _next_batch(self, fid):
        """Up to max_rhs RHS of field `fid` sharing one tolerance and one mass,
        in arrival order (caller holds the lock)."""
        batch = []
        tol = m0 = None
        for req in self._pending:
            if req.field_id != fid or req.next_rhs >= req.k:
                continue
            if tol is None:
                tol, m0 = req.tol, req.m0
            if req.tol != tol or req.m0 != m0:
                continue
            while req.next_rhs < req.k and len(batch) < self.max_rhs:
                batch.append((req, req.next_rhs))
                req.next_rhs += 1
            if len(batch) == self.max_rhs:
                break
        return batch, tol, m0

    def _dispatch(self):
        while True:
            with self._cv:
                while not self._runnable():
                    if self._closed and not self._pending:
                        return
                    self._cv.wait(timeout=0.05)
                started = 0
                for fid in self._runnable():
                    if fid not in self._resident and not self._admit(fid):
                        continue
                    self._busy.add(fid)
                    w = threading.Thread(target=self._work, args=(fid,), name="dd-field-%s" % (fid,), daemon=True)
                    self._workers[fid] = w
                    w.start()
                    started += 1
                if not started:
                    # every runnable field waits for memory: sleep until a worker
                    # finishes (it notifies) instead of polling
                    self._cv.wait(timeout=0.05)

    def _runnable(self):
        out = []
        for req in self._pending:
            fid = req.field_id
            if req.next_rhs < req.k and fid not in self._busy and fid not in out:
                out.append(fid)
        return out

    def _deliver(self, req, q, x, st, t):
        """Record the result of RHS q of req (caller holds the lock)."""
        req.x[q] = x.cpu() if (self.results_on_host and hasattr(x, "cpu")) else x
        req.stats[q] = st
        req.done += 1
        self._solved += 1
        if req.done == req.k:
            self._pending.remove(req)
            self._latency.append(t - req.t_submit)
            self._t_last = t
            xs, req.x = _stack(req.x), None
            req.rhs = None
            req.future.set_result((xs, req.stats))

    def _next_rhs(self, fid, m0):
        """The next queued RHS of field `fid` at mass m0 (any mass if None), in
        arrival order (caller holds the lock)."""
        for req in self._pending:
            if req.field_id != fid or req.next_rhs >= req.k:
                continue
            if m0 is not None and req.m0 != m0:
                continue
            q = req.next_rhs
            req.next_rhs += 1
            return req, q
        return None

    def _work_stream(self, fid, solver):
        """Continuous batching: refill every finished slot between restart
        cycles with the next queued RHS of this field (one mass at a time:
        the mass may change only when no slot runs)."""
        slots = [None] * self.max_rhs
        mass = None
        while True:
            with self._cv:
                self._resident.move_to_end(fid)
                running = any(sl is not None for sl in slots)
                if not running:
                    mass = None
                new = []
                for i in range(self.max_rhs):
                    if slots[i] is not None:
                        continue
                    nxt = self._next_rhs(fid, mass)
                    if nxt is None:
                        break
                    slots[i] = nxt
                    mass = nxt[0].m0
                    new.append(i)
            if not running and not new:
                return
            if new and not running and mass is not None and getattr(solver, "m0", mass) != mass:
                solver.set_mass(mass)
            for i in new:
                req, q = slots[i]
                solver.stream_load(i, req.rhs[q], req.tol)
            states, _ = solver.stream_cycle()
            done = []
            for i, stt in enumerate(states):
                if slots[i] is not None and stt in (solver.SLOT_CONVERGED, solver.SLOT_STOPPED):
                    x, st = solver.stream_take(i, allow_noconv=True)
                    done.append((slots[i], x, st))
                    slots[i] = None
            if done:
                t = self.clock()
                with self._cv:
                    for (req, q), x, st in done:
                        self._deliver(req, q, x, st, t)

    def _work(self, fid):
        """Worker of one field: set up if needed, then solve the field's queued
        RHS until none is left (continuous batching when the backend offers it,
        else whole batches; both return after their stream has finished)."""
        try:
            with self._cv:
                solver = self._resident.get(fid)
            if solver is None:
                try:
                    solver = self._factory(self._fields[fid])
                except BaseException:
                    with self._cv:
                        self._reserved.pop(fid, None)
                    raise
                # account what the setup really holds once it is known
                used = getattr(solver, "device_bytes", None)
                held = max(self._fields[fid].est_bytes, int(used()) if callable(used) else 0)
                with self._cv:
                    self._reserved.pop(fid, None)
                    self._resident[fid] = solver
                    self._resident_bytes[fid] = held
                    self.admitted += 1
                    self._trim(keep=fid)
            if hasattr(solver, "stream_cycle"):
                self._work_stream(fid, solver)
                return
            while True:
                with self._cv:
                    self._resident.move_to_end(fid)
                    batch, tol, m0 = self._next_batch(fid)
                if not batch:
                    break
                if m0 is not None and getattr(solver, "m0", m0) != m0:
                    solver.set_mass(m0)
                B = _stack([req.rhs[q] for req, q in batch])
                X, st = solver.solve_batch(B, tol)
                t = self.clock()
                with self._cv:
                    for i, (req, q) in enumerate(batch):
                        self._deliver(req, q, X[i], st[i], t)
        except BaseException as e:  # fail the requests of this field, keep serving others
            with self._cv:
                for req in [r for r in self._pending if r.field_id == fid]:
                    self._pending.remove(req)
                    if not req.future.done():
                        req.future.set_exception(e)
        finally:
            with self._cv:
                self._busy.discard(fid)
                self._cv.notify_all()
