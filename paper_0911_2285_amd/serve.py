"""Serving loop over several resident operators: continuous batching of
solve requests, deflation spaces grown online, admission by device-memory
budget, latency records.

Each operator keeps its gauge field and its deflation space on the device.
The first requests of an operator are solved by eigBiCG one at a time
(Alg. Incremental eigBiCG, step 2: each absorbs nev pairs), on a worker
thread per operator so that the loop keeps stepping the other operators'
sessions meanwhile; later requests go
to the operator's session (the library's eb_session), which batches them as
slots of the multi-RHS BiCGStab with their starts deflated by the space as it
is when they start (step 3).  Requests that arrive while others run are
admitted as slots and device memory free up, and the sessions of different
operators run on their own streams, so their work overlaps on the device.

This module schedules only: every solve runs in the HIP library.
"""
from __future__ import annotations

import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import ebicg


@dataclass
class Request:
    rid: int
    op: int          # index of the operator
    arrival: float   # seconds after the start of the run
    b: object        # host tensor, complex128 canonical spinor (pinned for an asynchronous upload)


@dataclass
class Result:
    rid: int
    op: int
    kind: str        # "eigbicg" (grows the space) or "session"
    arrival: float
    start: float     # admission time
    finish: float    # time the host saw the result
    status: str
    stats: dict
    K: int           # size of the operator's deflation space at admission
    x: object = None

    @property
    def latency(self):
        return self.finish - self.arrival


@dataclass
class OperatorSpec:
    op: object                 # ebicg.Operator
    grow: int = 0              # requests solved by eigBiCG first
    nev: int = 8
    m: int = 24
    slots: int = 8


@dataclass
class _Active:
    req: Request
    b: object
    x: object
    start: float
    K: int
    nbytes: int = field(default=0)


class Server:
    """Runs a stream of requests over the given operators.

    inner / tol / maxiter / chunk / graph: the sessions' parameters (eb_session_params);
    hbm_budget: device bytes the server may hold (operators, sessions and the
    requests' b and x); a request waits while it would exceed it."""

    def __init__(self, specs, inner="fp32", tol=1e-10, maxiter=20000, chunk=8, hbm_budget=None,
                 keep_solutions=False, graph=True, backend=None):
        self.eb = backend if backend is not None else ebicg   # the library binding (tests pass a stand-in)
        self.specs = list(specs)
        self.tol = float(tol)
        self.maxiter = int(maxiter)
        self.budget = hbm_budget
        self.keep = keep_solutions
        self.streams = [self._new_stream() for _ in self.specs]
        self.sessions = []
        for sp, st in zip(self.specs, self.streams):
            self.sessions.append(self.eb.Session(sp.op, slots=sp.slots, inner=inner, tol=tol, maxiter=maxiter,
                                                 chunk=chunk, graph=graph, stream=st))
        self.grow_left = [sp.grow for sp in self.specs]
        self.max_resident = 0
        self.deferred = 0   # admissions postponed by the memory budget
        # growth solves run on a worker per operator; while one runs, its
        # operator is not queried (its buffers may be growing): the last
        # measured size stands in for it
        self._pool = ThreadPoolExecutor(max_workers=max(1, len(self.specs)))
        self._growing = [None] * len(self.specs)
        self._op_bytes = [self.eb.op_device_bytes(sp.op) for sp in self.specs]

    def resident_bytes(self):
        for i, sp in enumerate(self.specs):
            if self._growing[i] is None:
                self._op_bytes[i] = self.eb.op_device_bytes(sp.op)
        return sum(self._op_bytes) + sum(s.info()["device_bytes"] for s in self.sessions)

    def _grow(self, i, b, x):
        sp = self.specs[i]
        try:
            st, _ = self.eb.eigbicg_solve(sp.op, b, x, sp.nev, sp.m, self.tol, maxiter=self.maxiter,
                                          stream=self.streams[i])
            return st, "EB_OK"
        except self.eb.EbicgError as e:
            return e.stats or {}, self.eb.STATUS.get(e.status, str(e.status))

    def _new_stream(self):
        import torch

        return torch.cuda.Stream()

    @staticmethod
    def _request_bytes(op):
        return 2 * 16 * op.N   # b and x, FP64 complex

    def _upload(self, i, req):
        import torch

        with torch.cuda.stream(self.streams[i]):
            b = req.b.to("cuda", non_blocking=True)
            x = torch.zeros_like(b)
        return b, x

    def _defl_K(self, i):
        return self.eb.defl_info(self.specs[i].op)[0]

    def run(self, requests):
        """Serve `requests` (arrival times relative to the call); returns the Results in finish order."""
        queue = sorted(requests, key=lambda r: r.arrival)
        waiting = [deque() for _ in self.specs]
        active = [dict() for _ in self.specs]
        results = []
        inflight = 0
        qi = 0
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0

        def fits(nbytes):
            if self.budget is None:
                return True
            return self.resident_bytes() + inflight + nbytes <= self.budget

        while qi < len(queue) or any(waiting) or any(active) or any(g is not None for g in self._growing):
            now = clock()
            while qi < len(queue) and queue[qi].arrival <= now:
                waiting[queue[qi].op].append(queue[qi])
                qi += 1
            blocked = False   # a request waits for memory
            admitted = False
            for i, sp in enumerate(self.specs):
                # growth phase: eigBiCG solves one at a time per operator, each
                # absorbing nev pairs, on the operator's worker
                if self.grow_left[i] > 0:
                    if self._growing[i] is None and waiting[i]:
                        nb = self._request_bytes(sp.op)
                        if not fits(nb):
                            self.deferred += 1
                            blocked = True
                        else:
                            req = waiting[i].popleft()
                            admitted = True
                            inflight += nb
                            self.max_resident = max(self.max_resident, self.resident_bytes() + inflight)
                            start, K = clock(), self._defl_K(i)
                            b, x = self._upload(i, req)
                            fut = self._pool.submit(self._grow, i, b, x)
                            self._growing[i] = (fut, req, x, start, K, nb)
                    continue
                sess = self.sessions[i]
                while waiting[i] and len(active[i]) < sp.slots:
                    nb = self._request_bytes(sp.op)
                    if not fits(nb):
                        self.deferred += 1
                        blocked = True
                        break
                    req = waiting[i].popleft()
                    b, x = self._upload(i, req)
                    if sess.admit(b, x, req.rid) is None:   # every slot of the session is busy
                        raise RuntimeError("session reports no free slot for an admitted request")
                    active[i][req.rid] = _Active(req, b, x, clock(), self._defl_K(i), nb)
                    inflight += nb
                    admitted = True
            if blocked and not any(active) and not any(g is not None for g in self._growing):
                raise RuntimeError("a waiting request does not fit the device-memory budget with nothing running")
            if admitted:
                self.max_resident = max(self.max_resident, self.resident_bytes() + inflight)
            # step only the sessions whose chunk has finished: a small operator's
            # slots turn over at its own pace, not at the largest operator's
            stepped = False
            for i, sess in enumerate(self.sessions):
                if active[i] and sess.ready():
                    sess.step()
                    stepped = True
            for i, g in enumerate(self._growing):
                if g is not None and g[0].done():
                    fut, req, x, start, K, nb = g
                    st, status = fut.result()
                    self._growing[i] = None
                    self.grow_left[i] -= 1
                    inflight -= nb
                    stepped = True
                    results.append(Result(req.rid, i, "eigbicg", req.arrival, start, clock(), status, st, K,
                                          x if self.keep else None))
            for i, sess in enumerate(self.sessions):
                for tag, status, st in sess.poll():
                    a = active[i].pop(tag)
                    inflight -= a.nbytes
                    results.append(Result(tag, i, "session", a.req.arrival, a.start, clock(), status, st, a.K,
                                          a.x if self.keep else None))
            if not any(active) and not any(waiting) and qi < len(queue) and all(g is None for g in self._growing):
                time.sleep(max(0.0, queue[qi].arrival - clock()))
            elif not stepped and not admitted:
                time.sleep(20e-6)   # every chunk still in flight: yield the core briefly
        return results

    def close(self):
        self._pool.shutdown(wait=True)
        for s in self.sessions:
            s.close()


def poisson_arrivals(n, rate, mix, seed):
    """n arrival times of a Poisson stream of the given rate (per second) and
    the operator of each request, drawn with probabilities `mix`."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    ops = rng.choice(len(mix), size=n, p=np.asarray(mix) / np.sum(mix))
    return t, ops


def latency_summary(results, t_first_arrival=0.0):
    """p50 / p99 latency (ms) and solves/s over the run (first arrival to last finish)."""
    lat = np.array([r.latency for r in results])
    span = max(r.finish for r in results) - t_first_arrival
    return {
        "requests": len(results),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "solves_per_s": len(results) / span if span > 0 else float("nan"),
    }
