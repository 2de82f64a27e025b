"""Serving loop with continuous batching of PCG solves.

Requests (a problem: mesh, coefficient field, partition, levels, tau; and
its loads) arrive over time.  The server

* admits a request for set-up when the library's own estimate of its device
  footprint (bddc_plan) fits the HBM budget beside everything admitted; set-ups
  run on worker threads, each with a stream of its own, so their host work
  overlaps the solves on the device;
* runs every set-up request's solve stepwise (bddc_solve_begin / _advance /
  _poll / _end) from one stepping thread, each on its own stream: between
  chunks of PCG iterations the stepper starts the solves of requests that
  became ready, so new work joins at iteration boundaries while other solves
  are in flight, and the kernels of all active solves share the device;
* batches requests of one problem (equal `key` and precision): with
  `resident`, set-up problems are kept (least recently used released for
  room), and the pending loads of a problem join one blocked solve of up to
  `max_cols` right-hand sides, whose launches read the operators once for all
  columns.  A request with more loads than that is solved in blocks.

Every numerical step runs in libbddc; this module only schedules calls.  A
request's result does not depend on what else is in flight: each handle has
its own device state and stream, every reduction has a fixed order, and a
blocked solve gives each column bitwise the result of solving it alone, so a
request's solution is bitwise the same alone and in the mix (tested).
"""

from __future__ import annotations

import threading
import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field
from typing import Hashable, List, Optional

import numpy as np

from .bddc import Solver, footprint


@dataclass(eq=False)   # requests compare by identity
class Request:
    prob: object                       # synth.Problem-like: nx, ny, coeff, part, nsub, levels, agglom, ...
    rhs: np.ndarray                    # (nrhs, n_free) host array
    rtol: float = 1e-8
    precision: str = "fp64"
    arrival: float = 0.0               # seconds, on the server's clock
    key: Optional[Hashable] = None     # requests with equal keys have the same problem (only the loads differ)
    # filled in by the server
    admitted: float = 0.0
    started: float = 0.0               # first PCG chunk enqueued
    done: float = 0.0
    iterations: List[int] = field(default_factory=list)
    solution: Optional[np.ndarray] = None
    footprint: int = 0
    batch: int = 1                     # requests solved together in one blocked solve
    reused: bool = False               # ran on a resident problem (no set-up)
    error: Optional[BaseException] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass(eq=False)
class _Problem:
    """A set-up (or setting-up) problem: its handle, stream and footprint."""
    key: object
    footprint: int
    solver: Optional[Solver] = None
    stream: object = None
    busy: bool = False                 # a solve or set-up is using it
    error: Optional[BaseException] = None


@dataclass(eq=False)
class _Solve:
    """One blocked solve in flight: requests of one problem and their loads."""
    prob: _Problem
    requests: List[Request]
    F: object = None                   # device loads (nrhs, n_free)
    blocks: List[tuple] = field(default_factory=list)   # column ranges still to solve
    cur: Optional[tuple] = None
    U: Optional[np.ndarray] = None
    iters: List[int] = field(default_factory=list)


class Server:
    """Continuous-batching solve server; see the module docstring.

    slots: solves in flight at once; setup_workers: concurrent set-ups;
    chunk: PCG iterations between scheduling points."""

    def __init__(self, slots: int = 4, hbm_budget: Optional[int] = None, resident: bool = False,
                 max_cols: int = 8, chunk: int = 8, setup_workers: int = 2):
        import torch
        self.torch = torch
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.8 * free)
        self.budget = int(hbm_budget)
        self.resident = resident
        self.max_cols = max_cols
        self.chunk = chunk
        self.slots = slots
        self.cv = threading.Condition()
        self.pending: List[Request] = []
        self.finished: List[Request] = []
        self.problems: "OrderedDict[object, _Problem]" = OrderedDict()   # least recently used first
        self.setup_queue: deque = deque()
        self.ready: deque = deque()          # (problem, requests) set up, waiting for the stepper
        self.in_flight = 0                   # bytes of problems admitted (resident or in use)
        self.active: List[_Solve] = []
        self.max_active = 0
        self.closing = False
        self.t0 = time.perf_counter()
        self._uid = 0
        self.workers = [threading.Thread(target=self._setup_worker, daemon=True) for _ in range(setup_workers)]
        self.stepper = threading.Thread(target=self._step_loop, daemon=True)
        for t in self.workers:
            t.start()
        self.stepper.start()

    # ---------------------------------------------------------------- public
    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request) -> Request:
        req.footprint = footprint(req.prob)
        with self.cv:
            if not req.arrival:
                req.arrival = self.now()
            self.pending.append(req)
            self._schedule()
            self.cv.notify_all()
        return req

    def drain(self):
        """Wait until every submitted request has finished."""
        with self.cv:
            while self.pending or self.active or self.setup_queue or self.ready or self._setting_up():
                self.cv.wait(0.05)

    def close(self):
        with self.cv:
            self.closing = True
            self.cv.notify_all()
        for t in self.workers:
            t.join()
        self.stepper.join()
        with self.cv:
            for p in self.problems.values():
                if p.solver is not None:
                    p.solver.close()
            self.problems.clear()

    def stats(self) -> dict:
        lat = np.array([r.latency for r in self.finished]) * 1e3
        span = max(r.done for r in self.finished) - min(r.arrival for r in self.finished)
        rhs = sum(r.rhs.shape[0] for r in self.finished)
        return {"requests": len(self.finished), "solves_per_s": len(self.finished) / span, "rhs_per_s": rhs / span,
                "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                "max_in_flight": self.max_active, "slots": self.slots, "hbm_budget": self.budget,
                "resident": self.resident, "reused": sum(r.reused for r in self.finished),
                "mean_batch": float(np.mean([r.batch for r in self.finished]))}

    # ------------------------------------------------------------- scheduling
    def _key(self, req: Request):
        if req.key is None:
            self._uid += 1
            return ("anon", self._uid)
        return (req.key, req.precision)

    def _setting_up(self) -> bool:
        return any(p.busy and p.solver is None and p.error is None for p in self.problems.values())

    def _gather(self, head: Request) -> List[Request]:
        """head and the pending requests of its problem (same precision and
        tolerance), in arrival order, up to max_cols right-hand sides."""
        batch, cols = [head], head.rhs.shape[0]
        if head.key is None:
            return batch
        for r in self.pending:
            if r is head or r.key != head.key or r.precision != head.precision or r.rtol != head.rtol:
                continue
            if cols + r.rhs.shape[0] > self.max_cols:
                break
            batch.append(r)
            cols += r.rhs.shape[0]
        return batch

    def _schedule(self):
        """Under the lock: move pending requests to set-up or to the stepper."""
        progress = True
        while progress and self.pending:
            progress = False
            for head in list(self.pending):
                hk = (head.key, head.precision) if head.key is not None else None
                p = self.problems.get(hk) if hk is not None else None
                if p is not None:
                    if p.busy:
                        continue                       # its problem is solving or being set up
                    batch = self._gather(head)
                    self._take(batch)
                    p.busy = True
                    self.problems.move_to_end(hk)
                    for r in batch:
                        r.reused = True
                    self.ready.append((p, batch))
                    progress = True
                    continue
                # a set-up: make room by releasing idle resident problems
                need = head.footprint
                while self.in_flight + need > self.budget:
                    idle = [k for k, e in self.problems.items() if not e.busy]
                    if not idle:
                        break
                    e = self.problems.pop(idle[0])
                    self.in_flight -= e.footprint
                    if e.solver is not None:
                        try:
                            e.solver.close()
                        except Exception:   # a failed release must not stop the server
                            pass
                nothing_running = not self.problems and not self.active
                if self.in_flight + need <= self.budget or nothing_running:
                    batch = self._gather(head)
                    self._take(batch)
                    key = self._key(head)
                    p = _Problem(key=key, footprint=need, busy=True)
                    self.problems[key] = p
                    self.in_flight += need
                    self.setup_queue.append((p, batch))
                    progress = True
                    break                              # admission is in arrival order
                break

    def _take(self, batch: List[Request]):
        taken = set(map(id, batch))
        self.pending = [r for r in self.pending if id(r) not in taken]
        now = self.now()
        for r in batch:
            r.admitted = now
            r.batch = len(batch)

    # ---------------------------------------------------------------- workers
    def _setup_worker(self):
        torch = self.torch
        while True:
            with self.cv:
                while not self.setup_queue and not self.closing:
                    self.cv.wait()
                if not self.setup_queue:
                    return
                p, batch = self.setup_queue.popleft()
            head = batch[0]
            try:
                stream = torch.cuda.Stream()
                with torch.cuda.stream(stream):
                    solver = Solver(head.prob, precision=head.precision, stream=stream)
                p.solver, p.stream = solver, stream
            except BaseException as e:  # reported on the requests
                p.error = e
            with self.cv:
                if p.error is not None:
                    self._finish_requests(batch, p.error)
                    self._drop(p)
                else:
                    self.ready.append((p, batch))
                self.cv.notify_all()

    def _finish_requests(self, batch: List[Request], err=None):
        now = self.now()
        for r in batch:
            r.done = now
            r.error = err
            self.finished.append(r)

    def _drop(self, p: _Problem):
        if self.problems.get(p.key) is p:
            del self.problems[p.key]
        self.in_flight -= p.footprint
        if p.solver is not None:
            try:
                p.solver.close()
            except Exception:   # a failed release must not stop the server
                pass
            p.solver = None

    def _release(self, p: _Problem, ok: bool):
        """After a solve: keep a resident problem, else release it."""
        if ok and self.resident and p.key[0] != "anon":
            p.busy = False
        else:
            self._drop(p)

    def _start(self, sv: _Solve):
        torch = self.torch
        F = np.concatenate([np.ascontiguousarray(r.rhs) for r in sv.requests], axis=0)
        with torch.cuda.stream(sv.prob.stream):
            sv.F = torch.tensor(F, dtype=torch.float64, device="cuda")
        n = F.shape[0]
        sv.blocks = [(c, min(n, c + self.max_cols)) for c in range(0, n, self.max_cols)]
        sv.U = np.empty_like(F)
        now = self.now()
        for r in sv.requests:
            r.started = now
        self._next_block(sv)

    def _next_block(self, sv: _Solve):
        c0, c1 = sv.blocks.pop(0)
        sv.cur = (c0, c1)
        f = sv.F[c0:c1]
        rtol = sv.requests[0].rtol
        sv.prob.solver.begin(f if c1 - c0 > 1 else f[0], rtol=rtol, stream=sv.prob.stream)
        sv.prob.solver.advance(self.chunk)

    def _step_loop(self):
        torch = self.torch
        while True:
            with self.cv:
                self._schedule()
                while self.ready and len(self.active) < self.slots:
                    p, batch = self.ready.popleft()
                    self.active.append(_Solve(prob=p, requests=batch))
                    self.active[-1].cur = None
                if not self.active:
                    if self.closing and not self.pending and not self.setup_queue and not self.ready:
                        return
                    self.cv.wait(0.002)
                    continue
                self.max_active = max(self.max_active, len(self.active))
                active = list(self.active)
            finished = []
            for sv in active:
                try:
                    if sv.cur is None:
                        self._start(sv)
                        continue
                    state = sv.prob.solver.poll()
                    if state == -1:
                        continue
                    if state == 0:
                        sv.prob.solver.advance(self.chunk)
                        continue
                    u, it, _ = sv.prob.solver.end()
                    c0, c1 = sv.cur
                    sv.U[c0:c1] = u.cpu().numpy().reshape(c1 - c0, -1)
                    sv.iters.extend(int(x) for x in it)
                    if sv.blocks:
                        self._next_block(sv)
                        continue
                    finished.append((sv, None))
                except BaseException as e:  # reported on the requests
                    finished.append((sv, e))
            if not finished:
                time.sleep(0.0002)
                continue
            with self.cv:
                for sv, err in finished:
                    self.active.remove(sv)
                    if err is None:
                        c = 0
                        for r in sv.requests:
                            n = r.rhs.shape[0]
                            r.solution = sv.U[c:c + n]
                            r.iterations = sv.iters[c:c + n]
                            c += n
                    self._finish_requests(sv.requests, err)
                    self._release(sv.prob, err is None)
                self._schedule()
                self.cv.notify_all()
