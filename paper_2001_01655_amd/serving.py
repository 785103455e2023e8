"""Continuous-batching request loop over the C ABI.

A request is a design problem: one mesh, supports, 1-4 load cases and a
sequence of density fields (successive design iterations).  For every density
the request needs K(rho) u_k = f_k solved for all its load cases, warm-started
from the previous design's displacements (the paper warm-starts each solve
with the previous optimisation iteration's solution, Sec. 4).

The loop:
  * admits queued requests whose arrival time has passed while a slot and
    enough HBM (tm_plan_bytes) are free; the hierarchy stays resident for all
    of the request's design iterations (tm_update_density between them);
  * keeps every admitted request on its own HIP stream (setup, design
    updates) and advances all running solves together with one batched call
    (tm_batch_iterate) on the server's stream, a few iterations at a time:
    the load cases of requests with the same level structure share every
    launch of an iteration, so small requests stop paying a launch each;
    results never mix across requests;
  * polls without blocking, retires finished solves, frees slot and memory
    when a request completes, and records latency from arrival to completion.

The device work goes through an engine object; `GpuEngine` drives libtopomg.
Tests can swap in another engine with the same methods to exercise the
scheduling logic alone.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                     # seconds after the start of the run
    nel: tuple
    fixed: np.ndarray
    loads: np.ndarray                  # (n_rhs, n_dof)
    densities: Callable[[int], np.ndarray]   # design index -> densities
    n_designs: int = 20
    material: dict = dataclasses.field(default_factory=dict)
    options: dict = dataclasses.field(default_factory=dict)

    @property
    def n_rhs(self) -> int:
        return int(self.loads.shape[0])


@dataclasses.dataclass
class Outcome:
    rid: int
    arrival: float
    admitted: float
    finished: float
    iters: List[List[int]]
    compliance: List[List[float]]
    status: List[int]
    u_last: Optional[object] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class _Slot:
    def __init__(self, req: Request, handle, stream, bytes_: int, admitted: float):
        self.req = req
        self.h = handle
        self.stream = stream
        self.bytes = bytes_
        self.design = 0
        self.state = None
        self.prep = None          # pending setup / update + begin (a future)
        self.u = None
        self.admitted = admitted
        self.iters: List[List[int]] = []
        self.comp: List[List[float]] = []
        self.status: List[int] = []


class _Now:
    """A finished 'future' for work done at once (no worker threads)."""

    def __init__(self, fn):
        self._v = fn()

    def done(self) -> bool:
        return True

    def result(self):
        return self._v


class Server:
    """Admission by HBM footprint, one stream per slot, batched iteration.

    workers > 0: a request's setup, each design update with the begin of its
    next solve, and the release of its hierarchy run on a pool of that many
    threads, so that a slow update (aggregation levels are rebuilt with
    host-side waits) never holds up the iterations of the other requests; the
    loop only collects what has finished.  workers = 0 does everything inline.

    gather: while chunks of other solves are still running, idle solves wait
    until they number at least gather times the running ones, so that they
    advance in fewer, larger grouped calls (the host cost of a call hardly
    depends on its size); with nothing running they advance at once.  0
    advances every idle solve at once; the default (infinite) advances all
    idle solves together once no chunk is running: the calls share one stream,
    so a solve's next chunk could not start before the running ones anyway."""

    def __init__(self, engine, hbm_budget: int, max_slots: int = 8, chunk: int = 4,
                 rtol: float = 1e-6, keep_solutions: bool = False, workers: int = 0,
                 gather: float = float("inf")):
        self.workers = int(workers)
        self.gather = float(gather)
        self.engine = engine
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk)
        self.rtol = float(rtol)
        self.keep = keep_solutions
        self.in_use = 0
        self.peak_in_use = 0
        self.queue_depth: List[int] = []

    # ------------------------------------------------------------------ slots
    def _later(self, fn):
        return self._pool.submit(fn) if self._pool is not None else _Now(fn)

    def _admit(self, req: Request, now: float) -> Optional[_Slot]:
        need = self.engine.plan_bytes(req)
        if need > self.budget:
            raise ValueError(f"request {req.rid} needs {need} bytes, more than the whole budget")
        if self.in_use + need > self.budget:
            return None
        stream = self.engine.new_stream()
        self.in_use += need
        self.peak_in_use = max(self.peak_in_use, self.in_use)
        s = _Slot(req, None, stream, need, now)

        def prepare():
            s.h = self.engine.setup(req, req.densities(0), stream)
            return self.engine.begin(s.h, s.req, self.rtol, s.u, s.stream)
        s.prep = self._later(prepare)
        return s

    def _next_design(self, s: _Slot):
        rho = s.req.densities(s.design)

        def prepare():
            self.engine.update(s.h, rho, s.stream)
            return self.engine.begin(s.h, s.req, self.rtol, s.u, s.stream)
        s.prep = self._later(prepare)

    def _finish_solve(self, s: _Slot):
        res = self.engine.end(s.state)
        s.state = None
        s.u = res.u
        s.iters.append(list(res.iters))
        s.comp.append(list(res.compliance))
        s.status.append(int(res.status))

    # ------------------------------------------------------------------ loop
    def run(self, requests: List[Request], clock: Optional[Callable[[], float]] = None) -> Dict:
        clock = clock or time.perf_counter
        pending = sorted(requests, key=lambda r: r.arrival)
        active: List[_Slot] = []
        done: List[Outcome] = []
        t0 = clock()
        n_solves = 0
        releasing = []                                        # (future, bytes)
        self._pool = None
        if self.workers > 0:
            from concurrent.futures import ThreadPoolExecutor
            self._pool = ThreadPoolExecutor(self.workers)
        try:
            while pending or active or releasing:
                now = clock() - t0
                # memory of released hierarchies returns to the budget once freed
                for fr in [x for x in releasing if x[0].done()]:
                    fr[0].result()
                    self.in_use -= fr[1]
                    releasing.remove(fr)
                # admission: arrived requests, in arrival order, while a slot and memory are free
                while pending and pending[0].arrival <= now and len(active) < self.max_slots:
                    s = self._admit(pending[0], now)
                    if s is None:
                        break
                    pending.pop(0)
                    active.append(s)
                self.queue_depth.append(sum(1 for r in pending if r.arrival <= now))
                # collect prepared solves, poll running ones without blocking
                idle = []
                running = 0
                for s in list(active):
                    if s.prep is not None:
                        if not s.prep.done():
                            continue
                        s.state = s.prep.result()
                        s.prep = None
                        idle.append(s)
                        continue
                    st = self.engine.poll(s.state)
                    if st == 1:                                   # every load case stopped
                        self._finish_solve(s)
                        n_solves += s.req.n_rhs
                        s.design += 1
                        if s.design < s.req.n_designs:
                            self._next_design(s)
                            if s.prep.done():                     # done inline: advance it now
                                s.state = s.prep.result()
                                s.prep = None
                                idle.append(s)
                        else:
                            fin = clock() - t0
                            done.append(Outcome(s.req.rid, s.req.arrival, s.admitted, fin, s.iters, s.comp,
                                                s.status, s.u if self.keep else None))
                            h = s.h
                            releasing.append((self._later(lambda h=h: self.engine.release(h)), s.bytes))
                            active.remove(s)
                    elif st == 0:                                 # chunk finished, keep going
                        idle.append(s)
                    else:
                        running += 1
                if idle and (running == 0 or len(idle) >= self.gather * running):
                    self.engine.batch_advance([s.state for s in idle], self.chunk)
                elif active or releasing:
                    time.sleep(5e-5)
                elif pending:
                    time.sleep(max(0.0, min(1e-3, pending[0].arrival - (clock() - t0))))
        finally:
            if self._pool is not None:
                self._pool.shutdown(wait=True)
        makespan = clock() - t0
        lat = np.array([o.latency for o in done]) if done else np.zeros(1)
        return {
            "outcomes": sorted(done, key=lambda o: o.rid),
            "makespan_s": makespan,
            "solves": n_solves,
            "solves_per_s": n_solves / makespan if makespan > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "peak_bytes": self.peak_in_use,
            "max_queue_depth": max(self.queue_depth) if self.queue_depth else 0,
        }


class GpuEngine:
    """Engine over libtopomg: one hierarchy per request, torch streams."""

    def __init__(self, **options):
        import torch
        from . import _lib as L
        from .solver import Hierarchy, tm_batch_iterate
        self.torch = torch
        self.L = L
        self.Hierarchy = Hierarchy
        self._batch = tm_batch_iterate
        self._stream = torch.cuda.Stream()     # grouped iterations of all requests
        self.options = options          # library options for every request (before the request's own)

    def _opts(self, req: Request) -> dict:
        o = dict(n_levels=0, max_coarse=1000, omega=0.5, nu_pre=1, nu_post=1, vcycle_fp=32, outer=0)
        o.update(self.options)
        o.update(req.options)
        return o

    def plan_bytes(self, req: Request) -> int:
        L = self.L
        return L.tm_plan_bytes(L.make_mesh(req.nel), L.default_options(**self._opts(req)), req.n_rhs)

    def new_stream(self):
        return self.torch.cuda.Stream()

    def setup(self, req: Request, rho, stream):
        with self.torch.cuda.stream(stream):
            H = self.Hierarchy(req.nel, rho, req.fixed, stream=stream, **req.material, **self._opts(req))
            H._f = self.torch.tensor(req.loads, device="cuda")
        return H

    def update(self, H, rho, stream):
        with self.torch.cuda.stream(stream):
            H.update_density(self.torch.tensor(rho, device="cuda"), stream=stream)

    def begin(self, H, req: Request, rtol: float, u0, stream):
        with self.torch.cuda.stream(stream):
            return H.begin(H._f, rtol, u0=u0, stream=stream)

    def poll(self, st) -> int:
        return st.poll()

    def batch_advance(self, states, k: int):
        self._batch(states, k, self._stream)

    def end(self, st):
        return st.end()

    def release(self, H):
        H.close()
