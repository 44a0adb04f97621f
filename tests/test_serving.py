"""Scheduling logic of the solve server, with an injected CPU backend (the
device path is covered by the GPU test at the end)."""
import threading
import time

import numpy as np
import pytest

from paper_1303_1377_amd import fields as F
from paper_1303_1377_amd.serving import Server, estimate_bytes


class FakeSolver:
    """x = 2 b; records the batch sizes and which fields run at the same time."""

    active = set()
    overlap = []
    lock = threading.Lock()

    def __init__(self, spec, delay=0.02):
        self.spec = spec
        self.batches = []
        self.delay = delay
        self.closed = False

    def solve_batch(self, B, tol):
        with FakeSolver.lock:
            FakeSolver.active.add(id(self))
            if len(FakeSolver.active) > 1:
                FakeSolver.overlap.append(len(FakeSolver.active))
        self.batches.append(len(B))
        time.sleep(self.delay)
        with FakeSolver.lock:
            FakeSolver.active.discard(id(self))
        return 2 * np.asarray(B), [dict(converged=1, tol=tol)] * len(B)

    def close(self):
        self.closed = True


def _server(budget, max_rhs=4, made=None):
    def factory(spec):
        s = FakeSolver(spec)
        if made is not None:
            made.append(s)
        return s

    return Server(budget_bytes=budget, max_rhs=max_rhs, solver_factory=factory)


def _rhs(dims, k, seed):
    return F.gaussian_spinor(dims, seed, nrhs=k)


def test_requests_share_batches_and_results_are_per_rhs():
    made = []
    srv = _server(1e12, max_rhs=4, made=made)
    dims = (4, 4, 4, 4)
    srv.add_field("a", dims, None, -0.4, 1.0)
    bs = [_rhs(dims, k, 10 + k) for k in (3, 2, 5)]
    futs = [srv.submit("a", b) for b in bs]
    for b, f in zip(bs, futs):
        x, st = f.result(timeout=10)
        assert np.array_equal(x, 2 * b) and len(st) == len(b)
    srv.close()
    assert len(made) == 1
    assert all(n <= 4 for n in made[0].batches) and sum(made[0].batches) == 10
    # RHS of different requests were batched together (10 RHS in fewer than 3+1+2 single-request batches)
    assert len(made[0].batches) <= 4
    st = srv.stats()
    assert st["requests"] == 3 and st["rhs_solved"] == 10 and st["p99_latency_s"] >= st["p50_latency_s"] > 0


def test_tolerances_are_not_mixed_in_a_batch():
    made = []
    srv = _server(1e12, max_rhs=8, made=made)
    dims = (4, 4, 4, 4)
    srv.add_field("a", dims, None, -0.4, 1.0)
    f1 = srv.submit("a", _rhs(dims, 2, 1), tol=1e-10)
    f2 = srv.submit("a", _rhs(dims, 2, 2), tol=1e-6)
    assert all(s["tol"] == 1e-10 for s in f1.result(timeout=10)[1])
    assert all(s["tol"] == 1e-6 for s in f2.result(timeout=10)[1])
    srv.close()


def test_budget_admission_and_lru_eviction():
    dims = (4, 4, 4, 4)
    one = estimate_bytes(dims, None, 4)
    made = []
    srv = _server(int(one * 1.5), max_rhs=4, made=made)   # room for one resident setup
    srv.add_field("a", dims, None, -0.4, 1.0)
    srv.add_field("b", dims, None, -0.4, 1.0)
    srv.submit("a", _rhs(dims, 1, 1)).result(timeout=10)
    assert srv.stats()["resident"] == ["a"]
    srv.submit("b", _rhs(dims, 1, 2)).result(timeout=10)
    st = srv.stats()
    assert st["resident"] == ["b"] and st["evicted"] == 1 and st["admitted"] == 2
    assert made[0].closed and not made[1].closed
    srv.close()


def test_setups_in_flight_respect_the_budget():
    """Setups being built hold their estimate: with room for 1.5 setups and a
    slow setup, three fields are never set up at once, and the bytes held
    (resident plus reserved) never exceed the budget."""
    dims = (4, 4, 4, 4)
    one = estimate_bytes(dims, None, 4)
    budget = int(one * 1.5)
    live = [0]
    peak = [0]
    lock = threading.Lock()
    srv_ref = []

    def factory(spec):
        with lock:
            live[0] += 1
            peak[0] = max(peak[0], live[0])
        st = srv_ref[0].stats()
        assert st["resident_bytes"] + st["reserved_bytes"] <= budget
        time.sleep(0.2)
        with lock:
            live[0] -= 1
        return FakeSolver(spec, delay=0.01)

    srv = Server(budget_bytes=budget, max_rhs=4, solver_factory=factory)
    srv_ref.append(srv)
    for f in ("a", "b", "c"):
        srv.add_field(f, dims, None, -0.4, 1.0)
    futs = [srv.submit(f, _rhs(dims, 2, i)) for i, f in enumerate(("a", "b", "c"))]
    samples = []
    while not all(f.done() for f in futs):
        st = srv.stats()
        samples.append(st["resident_bytes"] + st["reserved_bytes"])
        time.sleep(0.005)
    for f in futs:
        f.result(timeout=10)
    srv.close()
    assert peak[0] == 1
    assert max(samples) <= budget


def test_field_above_budget_is_refused():
    srv = _server(1e6)
    with pytest.raises(ValueError):
        srv.add_field("big", (16, 16, 16, 16), None, 0.0, 1.0)
    srv.close()


def test_fields_run_concurrently():
    FakeSolver.overlap.clear()
    srv = _server(1e12, max_rhs=2)
    dims = (4, 4, 4, 4)
    for f in ("a", "b", "c"):
        srv.add_field(f, dims, None, -0.4, 1.0)
    futs = [srv.submit(f, _rhs(dims, 4, i)) for i, f in enumerate(("a", "b", "c"))]
    for f in futs:
        f.result(timeout=10)
    srv.close()
    assert FakeSolver.overlap, "batches of different fields never overlapped"


def test_backend_failure_fails_only_that_field():
    dims = (4, 4, 4, 4)

    def factory(spec):
        if spec.m0 > 0:
            raise RuntimeError("setup failed")
        return FakeSolver(spec)

    srv = Server(budget_bytes=1e12, max_rhs=4, solver_factory=factory)
    srv.add_field("bad", dims, None, 0.5, 1.0)
    srv.add_field("good", dims, None, -0.4, 1.0)
    fb = srv.submit("bad", _rhs(dims, 1, 1))
    fg = srv.submit("good", _rhs(dims, 1, 2))
    with pytest.raises(RuntimeError):
        fb.result(timeout=10)
    assert fg.result(timeout=10)[0].shape == (1, 256, 4, 3)
    srv.close()


def test_masses_are_not_mixed_in_a_batch():
    """Requests at two masses on one field: every batch holds one mass, the
    resident setup is moved (set_mass) only when the mass changes, and no
    second setup is made."""
    masses = []

    class MassSolver(FakeSolver):
        def __init__(self, spec):
            super().__init__(spec)
            self.m0 = spec.m0
            self.calls = []

        def set_mass(self, m0):
            self.m0 = m0
            self.calls.append(m0)

        def solve_batch(self, B, tol):
            masses.append((self.m0, len(B)))
            return super().solve_batch(B, tol)

    made = []

    def factory(spec):
        s = MassSolver(spec)
        made.append(s)
        return s

    srv = Server(budget_bytes=1e12, max_rhs=4, solver_factory=factory)
    srv.add_field("f", (4, 4, 4, 4), None, -0.4, 1.0)
    futs = [srv.submit("f", np.ones((2, 256, 4, 3)), m0=(-0.4 if i % 2 == 0 else -0.3)) for i in range(6)]
    res = [f.result(timeout=10) for f in futs]
    srv.close()
    assert len(made) == 1
    assert all(np.allclose(x, 2.0) for x, _ in res)
    # three requests of 2 RHS per mass: batches of at most 4, never mixed
    assert sum(k for m, k in masses if m == -0.4) == 6 and sum(k for m, k in masses if m == -0.3) == 6
    assert all(k <= 4 for _, k in masses)
    assert len(made[0].calls) <= len(masses)


class FakeStreamSolver:
    """Continuous-batching backend: a RHS b needs 1 + round(|b[0,0,0]| * 4)
    restart cycles (capped at 6) and its solution is 2 b; records how many
    slots run in each cycle and the order in which RHS finish."""

    SLOT_FREE, SLOT_RUNNING, SLOT_CONVERGED, SLOT_STOPPED = 0, 1, 2, 3

    def __init__(self, spec, max_rhs):
        self.spec = spec
        self.m0 = spec.m0
        self.slots = [None] * max_rhs     # [b, cycles left]
        self.state = [0] * max_rhs
        self.occupancy = []
        self.finished = []

    def stream_load(self, i, b, tol):
        assert self.state[i] == 0
        b = np.asarray(b)
        self.slots[i] = [b, 1 + min(5, int(round(abs(b.reshape(-1)[0]) * 4)))]
        self.state[i] = 1

    def stream_cycle(self):
        self.occupancy.append(sum(1 for st in self.state if st == 1))
        time.sleep(0.002)
        for i, sl in enumerate(self.slots):
            if self.state[i] == 1:
                sl[1] -= 1
                if sl[1] == 0:
                    self.state[i] = 2
        return list(self.state), [dict(converged=st == 2) for st in self.state]

    def stream_take(self, i, allow_noconv=False):
        assert self.state[i] in (2, 3)
        b = self.slots[i][0]
        self.finished.append(float(b.reshape(-1)[0]))
        self.slots[i] = None
        self.state[i] = 0
        return 2 * b, dict(converged=True)

    def set_mass(self, m0):
        assert all(st != 1 for st in self.state), "mass changed while slots run"
        self.m0 = m0

    def close(self):
        pass


def test_continuous_batching_refills_finished_slots():
    """A slot whose RHS finished takes the next queued RHS at the following
    restart cycle, while the other slots keep running: short solves queued
    behind a long one finish before it, every cycle with queued work keeps
    all slots busy, and each result is the RHS's own."""
    made = []

    def factory(spec):
        s = FakeStreamSolver(spec, 4)
        made.append(s)
        return s

    srv = Server(budget_bytes=1e12, max_rhs=4, solver_factory=factory)
    dims = (4, 4, 4, 4)
    srv.add_field("f", dims, None, -0.4, 1.0)
    long_b = np.full((1, 256, 4, 3), 1.25)          # 6 cycles
    short = [np.full((1, 256, 4, 3), 0.01 * (i + 1)) for i in range(9)]   # 1 cycle each
    futs = [srv.submit("f", long_b)] + [srv.submit("f", b) for b in short]
    res = [f.result(timeout=10) for f in futs]
    srv.close()
    assert np.array_equal(res[0][0], 2 * long_b)
    for b, (x, _) in zip(short, res[1:]):
        assert np.array_equal(x, 2 * b)
    s = made[0]
    assert s.finished[-1] == 1.25            # the long solve ends last
    # 10 RHS in 4 slots: the short ones stream through the three slots the long one leaves
    assert len(s.occupancy) <= 6 and max(s.occupancy) == 4


def test_continuous_batching_keeps_one_mass_per_cycle():
    made = []

    def factory(spec):
        s = FakeStreamSolver(spec, 4)
        made.append(s)
        return s

    srv = Server(budget_bytes=1e12, max_rhs=4, solver_factory=factory)
    srv.add_field("f", (4, 4, 4, 4), None, -0.4, 1.0)
    futs = [srv.submit("f", np.full((2, 256, 4, 3), 0.3), m0=(-0.4 if i % 2 == 0 else -0.3)) for i in range(6)]
    res = [f.result(timeout=10) for f in futs]
    srv.close()
    assert all(np.allclose(x, 0.6) for x, _ in res)


@pytest.mark.gpu
def test_served_results_equal_solo_solves():
    """Two resident fields of different sizes, requests of 1..5 RHS arriving
    while others run: each result equals the solo solve of the same RHS on a
    setup of its own (to 1e-12: batched RHS advance exactly as single solves),
    and meets the 1e-10 true residual."""
    import torch

    import oracle as O
    import paper_1303_1377_amd as G

    specs = {"small": ((4, 4, 4, 4), 0, -0.4), "large": ((8, 8, 8, 8), 1, -0.25)}
    kw = dict(levels=2, n_tv=[8], agg=[(2, 2, 2, 2)], sap=[(2, 2, 2, 2)], mr_steps=[4], n_inv=2, outer_restart=20)
    srv = Server(budget_bytes=50e9, max_rhs=4)
    U = {}
    for name, (dims, seed, m0) in specs.items():
        U[name] = F.make_gauge(dims, 0.3, seed)
        srv.add_field(name, dims, U[name], m0, 1.0, params=G.default_params(**kw))
    rng = np.random.default_rng(0)
    reqs = []
    for i in range(8):
        name = ("small", "large")[i % 2]
        dims = specs[name][0]
        k = int(rng.integers(1, 6))
        b = F.gaussian_spinor(dims, 300 + i, nrhs=k)
        reqs.append((name, b, srv.submit(name, torch.as_tensor(b).to("cuda"))))
        time.sleep(0.01 * (i % 3))
    out = [(name, b, f.result(timeout=120)) for name, b, f in reqs]
    st = srv.stats()
    srv.close()
    print("serving stats", st, flush=True)
    for name, (dims, seed, m0) in specs.items():
        solo = G.Solver(dims, U[name], m0, 1.0)
        solo.setup(params=G.default_params(max_rhs=4, **kw))
        orc = O.Oracle(dims, U[name], m0, 1.0)
        for nm, b, (x, sts) in out:
            if nm != name:
                continue
            x = x.cpu().numpy()
            for q in range(len(b)):
                xs, _ = solo.solve(b[q], 1e-10)
                xs = xs.cpu().numpy()
                assert np.linalg.norm(x[q] - xs) <= 1e-12 * np.linalg.norm(xs)
                r = b[q] - orc.apply(x[q])
                assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b[q]) and sts[q]["converged"]
        solo.close()
    assert st["requests"] == 8 and st["p99_latency_s"] > 0


@pytest.mark.gpu
def test_served_masses_meet_their_residuals():
    """Requests at two masses on one resident 8^4 setup: each result meets
    the 1e-10 true residual of the operator at its own mass (the setup is
    shifted, not rebuilt), and equals the solve of a setup moved to that mass
    with dd_set_mass directly."""
    import torch

    import oracle as O
    import paper_1303_1377_amd as G

    dims = (8, 8, 8, 8)
    U = F.make_gauge(dims, 0.3, 2)
    kw = dict(levels=2, n_tv=[8], agg=[(2, 2, 2, 2)], sap=[(2, 2, 2, 2)], mr_steps=[4], n_inv=2, outer_restart=20)
    masses = (-0.25, -0.2)
    srv = Server(budget_bytes=50e9, max_rhs=4)
    srv.add_field("f", dims, U, masses[0], 1.0, params=G.default_params(**kw))
    reqs = []
    for i in range(6):
        m = masses[i % 2]
        b = F.gaussian_spinor(dims, 600 + i, nrhs=2)
        reqs.append((m, b, srv.submit("f", torch.as_tensor(b).to("cuda"), m0=m)))
    out = [(m, b, f.result(timeout=120)) for m, b, f in reqs]
    srv.close()
    orc = {m: O.Oracle(dims, U, m, 1.0) for m in masses}
    solo = G.Solver(dims, U, masses[0], 1.0)
    solo.setup(params=G.default_params(max_rhs=4, **kw))
    for m, b, (x, sts) in out:
        x = x.cpu().numpy()
        solo.set_mass(m)
        for q in range(len(b)):
            r = b[q] - orc[m].apply(x[q])
            assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b[q]) and sts[q]["converged"]
            xs, _ = solo.solve(b[q], 1e-10)
            xs = xs.cpu().numpy()
            assert np.linalg.norm(x[q] - xs) <= 1e-12 * np.linalg.norm(xs)
    solo.close()


@pytest.mark.gpu
def test_stream_slots_refilled_match_solo_solves():
    """dd_stream_*: six right-hand sides through three slots, each finished
    slot refilled with the next RHS between restart cycles; every result
    equals the single solve of its RHS (1e-12) and meets its true residual,
    and dd_solve is refused while slots are in use."""
    import oracle as O
    import paper_1303_1377_amd as G

    dims = (8, 8, 8, 8)
    U = F.make_gauge(dims, 0.3, 4)
    kw = dict(levels=2, n_tv=[8], agg=[(2, 2, 2, 2)], sap=[(2, 2, 2, 2)], mr_steps=[4], n_inv=2, outer_restart=5)
    s = G.Solver(dims, U, -0.25, 1.0)
    s.setup(params=G.default_params(max_rhs=3, **kw))
    solo = G.Solver(dims, U, -0.25, 1.0)
    solo.setup(params=G.default_params(max_rhs=3, **kw))
    orc = O.Oracle(dims, U, -0.25, 1.0)
    bs = [F.gaussian_spinor(dims, 900 + i) * (10.0 ** (-(i % 3))) for i in range(6)]
    queue = list(range(6))
    slot_of = [None] * 3
    results = {}
    cycles = 0
    while queue or any(v is not None for v in slot_of):
        for i in range(3):
            if slot_of[i] is None and queue:
                q = queue.pop(0)
                s.stream_load(i, bs[q], 1e-10)
                slot_of[i] = q
        if cycles == 0:
            with pytest.raises(G.DDError) as ei:
                s.solve(bs[0], 1e-10)
            assert ei.value.code == -5
        states, _ = s.stream_cycle()
        cycles += 1
        for i, stt in enumerate(states):
            if slot_of[i] is not None and stt in (s.SLOT_CONVERGED, s.SLOT_STOPPED):
                x, st = s.stream_take(i)
                results[slot_of[i]] = (x.cpu().numpy(), st)
                slot_of[i] = None
        assert cycles < 200
    for q, b in enumerate(bs):
        x, st = results[q]
        xs, sts = solo.solve(b, 1e-10)
        xs = xs.cpu().numpy()
        assert st["converged"] and st["outer_iters"] == sts["outer_iters"]
        assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)
        r = b - orc.apply(x)
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b)
    s.close()
    solo.close()
