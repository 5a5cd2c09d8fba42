"""Host logic of the serving loop (paper_0911_2285_amd/serve.py) on the CPU,
with a stand-in for the library binding: growth of each operator's space by
its first requests, admission by memory budget, and the arrival generator.
The GPU path of the same loop is covered in test_gpu_serve.py."""
import numpy as np
import pytest

from paper_0911_2285_amd import serve


class _Err(RuntimeError):
    def __init__(self, status, stats=None):
        super().__init__(status)
        self.status, self.stats = status, stats


class _Op:
    def __init__(self, N, nbytes):
        self.N, self.bytes, self.K = N, nbytes, 0


class _Req:
    """Stands in for a source tensor: the request finishes after `chunks` steps."""

    def __init__(self, chunks):
        self.chunks = chunks


class _Session:
    def __init__(self, op, slots, **kw):
        self.op, self.slots = op, slots
        self.active = {}   # tag -> chunks left
        self.done = []
        self.max_busy = 0

    def admit(self, b, x, tag):
        if len(self.active) >= self.slots:
            return None
        self.active[tag] = b.chunks
        self.max_busy = max(self.max_busy, len(self.active))
        return len(self.active) - 1

    def ready(self):
        return True

    def step(self):
        for tag in list(self.active):
            self.active[tag] -= 1
            if self.active[tag] <= 0:
                del self.active[tag]
                self.done.append((tag, "EB_OK", {"iters": 1, "true_rel_resid": 0.0}))

    def poll(self):
        out, self.done = self.done, []
        return out

    def info(self):
        return {"free": self.slots - len(self.active), "busy": len(self.active), "done": len(self.done),
                "device_bytes": 1000}

    def close(self):
        pass


class _Backend:
    EbicgError = _Err
    STATUS = {0: "EB_OK"}
    Session = _Session

    def __init__(self):
        self.sessions = []
        self.eig_calls = []

    @staticmethod
    def op_device_bytes(op):
        return op.bytes

    @staticmethod
    def defl_info(op):
        return op.K, None

    def eigbicg_solve(self, op, b, x, nev, m, tol, maxiter, stream):
        self.eig_calls.append(op)
        op.K += nev
        return {"iters": 1, "true_rel_resid": 0.0}, None


class _Server(serve.Server):
    def _new_stream(self):
        return None

    def _upload(self, i, req):
        return req.b, object()


def _reqs(n, ops, chunks=3, t=None):
    t = np.zeros(n) if t is None else t
    return [serve.Request(i, ops[i], float(t[i]), _Req(chunks)) for i in range(n)]


def test_growth_requests_come_first_then_sessions_use_the_space():
    be = _Backend()
    ops = [_Op(96, 10_000), _Op(192, 20_000)]
    specs = [serve.OperatorSpec(o, grow=2, nev=4, m=16, slots=4) for o in ops]
    srv = _Server(specs, backend=be)
    which = [0, 1, 0, 1, 0, 0, 1, 1, 0, 1]
    res = srv.run(_reqs(10, which))
    assert len(res) == 10 and all(r.status == "EB_OK" for r in res)
    kinds = {r.rid: r.kind for r in res}
    for o in (0, 1):
        rids = [i for i, w in enumerate(which) if w == o]
        assert [kinds[i] for i in rids[:2]] == ["eigbicg", "eigbicg"]
        assert all(kinds[i] == "session" for i in rids[2:])
    assert all(r.K == 8 for r in res if r.kind == "session")
    assert [r.K for r in res if r.kind == "eigbicg"].count(0) == 2   # the first solve of each operator
    assert ops[0].K == 8 and ops[1].K == 8


def test_memory_budget_defers_admissions_and_caps_requests_in_flight():
    be = _Backend()
    op = _Op(1000, 50_000)
    per_req = 2 * 16 * op.N
    specs = [serve.OperatorSpec(op, grow=0, slots=8)]
    srv = _Server(specs, backend=be)
    resident = srv.resident_bytes()
    srv.budget = resident + 2 * per_req
    res = srv.run(_reqs(9, [0] * 9, chunks=3))
    assert len(res) == 9
    assert srv.deferred > 0 and srv.max_resident <= srv.budget
    assert srv.sessions[0].max_busy == 2


def test_a_request_that_can_never_fit_raises_instead_of_waiting_forever():
    be = _Backend()
    op = _Op(1000, 50_000)
    srv = _Server([serve.OperatorSpec(op, grow=0, slots=4)], backend=be)
    srv.budget = srv.resident_bytes() + 16 * op.N   # half of one request
    with pytest.raises(RuntimeError, match="budget"):
        srv.run(_reqs(2, [0, 0]))
    srv2 = _Server([serve.OperatorSpec(_Op(1000, 50_000), grow=1, slots=4)], backend=be)
    srv2.budget = srv2.resident_bytes() + 16 * 1000
    with pytest.raises(RuntimeError, match="budget"):
        srv2.run(_reqs(1, [0]))


def test_arrivals_wait_for_their_time():
    be = _Backend()
    op = _Op(10, 100)
    srv = _Server([serve.OperatorSpec(op, grow=0, slots=2)], backend=be)
    t = np.array([0.0, 0.05, 0.10])
    res = srv.run(_reqs(3, [0, 0, 0], chunks=1, t=t))
    for r in res:
        assert r.start >= r.arrival - 1e-9 and r.finish >= r.start and r.latency >= 0


def test_poisson_arrivals_rate_and_mix():
    t, ops = serve.poisson_arrivals(20000, rate=50.0, mix=[0.5, 0.35, 0.15], seed=7)
    t2, ops2 = serve.poisson_arrivals(20000, rate=50.0, mix=[0.5, 0.35, 0.15], seed=7)
    assert np.array_equal(t, t2) and np.array_equal(ops, ops2)
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 1 / 50.0) < 0.03 / 50.0
    frac = np.bincount(ops, minlength=3) / len(ops)
    assert np.allclose(frac, [0.5, 0.35, 0.15], atol=0.015)


def test_latency_summary_percentiles():
    res = [serve.Result(i, 0, "session", 0.0, 0.0, 0.001 * (i + 1), "EB_OK", {}, 0) for i in range(100)]
    s = serve.latency_summary(res)
    assert s["requests"] == 100
    assert abs(s["p50_ms"] - 50.5) < 1e-9 and abs(s["p99_ms"] - 99.01) < 1e-9
    assert abs(s["solves_per_s"] - 1000.0) < 1e-9
