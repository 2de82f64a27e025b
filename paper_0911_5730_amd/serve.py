"""Serving loop: solve requests admitted onto concurrent slots, with resident
problems and merged right-hand sides.

Each slot is a host thread with a HIP stream of its own.  A request carries a
problem (mesh, coefficient field, partition, levels, tau) and its loads; a
slot takes the oldest request it can run:

* a request whose problem is resident (set up earlier and kept, `key` equal)
  runs on that handle without a new set-up, and the pending requests of the
  same problem (same precision and tolerance) join it, up to `max_cols`
  right-hand sides in one blocked solve: every launch of that solve reads the
  problem's operators once for all of them;
* otherwise the request is admitted when the estimated device footprint of
  everything resident or running stays within the HBM budget (idle resident
  problems are released, least recently used first, to make room; at least
  one request is always admitted, so none starves); it is set up on the slot
  and, with `resident`, kept for later requests of its problem.

One request's host set-up overlaps the kernels of the others, and their
kernels share the device.  Every numerical step runs in libbddc
(bddc_setup / bddc_solve / bddc_destroy); this module only schedules the
calls.  Results do not depend on what else is in flight: each handle has its
own device state, every reduction has a fixed order, and a blocked solve gives
every column bitwise the result of solving it alone, so a request's solution
is bitwise the same alone and in the mix (tested).
"""

from __future__ import annotations

import threading
import time
from collections import OrderedDict
from dataclasses import dataclass, field
from typing import Hashable, List, Optional

import numpy as np

from .bddc import Solver


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


def footprint_bytes(prob) -> int:
    """Device bytes a request will hold, estimated from its sizes: the dense
    local matrices of every level-1 substructure dominate (the deeper levels
    are a small fraction), plus the vectors and interface data."""
    nfree = (prob.nx - 1) * (prob.ny - 1)
    per = nfree / max(1, prob.nsub)
    nloc = per + 4.0 * np.sqrt(per) + 4.0            # interior plus the substructure's boundary layer
    return int(8.0 * prob.nsub * nloc * nloc * 1.25 + 200.0 * nfree)


@dataclass(eq=False)
class _Resident:
    solver: Optional[Solver]           # None while its set-up runs
    footprint: int
    busy: bool = False


class Server:
    """Slots of concurrent set-up + solve; see the module docstring."""

    def __init__(self, slots: int = 2, hbm_budget: Optional[int] = None, resident: bool = False,
                 max_cols: int = 8):
        import torch
        self.torch = torch
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.8 * free)
        self.budget = int(hbm_budget)
        self.resident = resident
        self.max_cols = max_cols
        self.cv = threading.Condition()
        self.pending: List[Request] = []
        self.finished: List[Request] = []
        self.handles: "OrderedDict[tuple, _Resident]" = OrderedDict()   # least recently used first
        self.in_flight = 0                 # bytes: resident problems and running set-ups
        self.active = 0                    # running solves
        self.max_active = 0
        self.closing = False
        self.t0 = time.perf_counter()
        self.threads = [threading.Thread(target=self._slot, args=(k,), daemon=True) for k in range(slots)]
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        for t in self.threads:
            t.start()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request) -> Request:
        req.footprint = footprint_bytes(req.prob)
        with self.cv:
            if not req.arrival:
                req.arrival = self.now()
            self.pending.append(req)
            self.cv.notify_all()
        return req

    @staticmethod
    def _hkey(req: Request):
        return None if req.key is None else (req.key, req.precision)

    def _gather(self, head: Request) -> List[Request]:
        """head and the pending requests of its problem (same precision and
        tolerance), in arrival order, up to max_cols right-hand sides."""
        batch, cols = [head], head.rhs.shape[0]
        hk = self._hkey(head)
        if hk is None:
            return batch
        for r in self.pending:
            if r is head or self._hkey(r) != hk or r.rtol != head.rtol:
                continue
            if cols + r.rhs.shape[0] > self.max_cols:
                break
            batch.append(r)
            cols += r.rhs.shape[0]
        return batch

    def _take(self):
        """The next work under the lock: (batch, resident entry or None), or None."""
        for head in self.pending:
            hk = self._hkey(head)
            if hk is not None and hk in self.handles:
                ent = self.handles[hk]
                if ent.busy:
                    continue                      # its problem is solving on another slot
                batch = self._gather(head)
                ent.busy = True
                self.handles.move_to_end(hk)
                return batch, ent
            # a set-up: make room by releasing idle resident problems
            need = head.footprint
            while self.in_flight + need > self.budget:
                idle = [k for k, e in self.handles.items() if not e.busy]
                if not idle:
                    break
                ent = self.handles.pop(idle[0])
                self.in_flight -= ent.footprint
                if ent.solver is not None:
                    try:
                        ent.solver.close()
                    except Exception:   # a failed release must not stop the slot
                        pass
            if self.active == 0 or self.in_flight + need <= self.budget:
                self.in_flight += need
                if self.resident and hk is not None:
                    # the other slots see the problem as busy while it is set up
                    self.handles[hk] = _Resident(None, need, busy=True)
                return self._gather(head), None
            return None                           # the oldest set-up waits for room
        return None

    def _slot(self, k: int):
        torch = self.torch
        stream = self.streams[k]
        while True:
            with self.cv:
                while True:
                    got = self._take()
                    if got is not None or (self.closing and not self.pending):
                        break
                    self.cv.wait()
                if got is None:
                    return
                batch, ent = got
                taken = set(map(id, batch))
                self.pending = [r for r in self.pending if id(r) not in taken]
                for r in batch:
                    r.admitted = self.now()
                    r.batch = len(batch)
                    r.reused = ent is not None
                self.active += 1
                self.max_active = max(self.max_active, self.active)
            head = batch[0]
            err = None
            keep = None
            try:
                with torch.cuda.stream(stream):
                    S = ent.solver if ent is not None else Solver(head.prob, precision=head.precision, stream=stream)
                    try:
                        F = np.concatenate([np.ascontiguousarray(r.rhs) for r in batch], axis=0)
                        # (nrhs, n_free) rows are the columns of the library's n_free x nrhs layout
                        f = torch.tensor(F, dtype=torch.float64, device="cuda")
                        u, it, _ = S.solve(f, rtol=head.rtol, stream=stream)
                        U = u.cpu().numpy()
                        c = 0
                        for r in batch:
                            n = r.rhs.shape[0]
                            r.solution = U[c:c + n]
                            r.iterations = [int(x) for x in it[c:c + n]]
                            c += n
                    finally:
                        if ent is None and self.resident and self._hkey(head) is not None:
                            keep = S
                        elif ent is None:
                            S.close()
            except BaseException as e:  # reported on the requests
                err = e
            with self.cv:
                now = self.now()
                for r in batch:
                    r.done = now
                    r.error = err
                    self.finished.append(r)
                hk = self._hkey(head)
                if ent is not None and err is not None:
                    # a failed solve leaves the handle in an unknown state:
                    # release it, later requests of the problem set it up anew
                    if self.handles.get(hk) is ent:
                        del self.handles[hk]
                    self.in_flight -= ent.footprint
                    try:
                        ent.solver.close()
                    except Exception:   # a failed release must not stop the slot
                        pass
                elif ent is not None:
                    ent.busy = False
                elif keep is not None and err is None:
                    ph = self.handles[hk]                  # the placeholder of the set-up
                    ph.solver, ph.busy = keep, False       # stays in flight
                else:
                    if keep is not None:
                        keep.close()
                    if self.resident and hk is not None and hk in self.handles and self.handles[hk].solver is None:
                        del self.handles[hk]
                    self.in_flight -= head.footprint
                self.active -= 1
                self.cv.notify_all()

    def drain(self):
        """Wait until every submitted request has finished."""
        with self.cv:
            while self.pending or self.active:
                self.cv.wait()

    def close(self):
        with self.cv:
            self.closing = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()
        with self.cv:
            for ent in self.handles.values():
                if ent.solver is not None:
                    ent.solver.close()
            self.handles.clear()

    def stats(self) -> dict:
        lat = np.array([r.latency for r in self.finished]) * 1e3
        span = max(r.done for r in self.finished) - min(r.arrival for r in self.finished)
        rhs = sum(r.rhs.shape[0] for r in self.finished)
        return {"requests": len(self.finished), "solves_per_s": len(self.finished) / span, "rhs_per_s": rhs / span,
                "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                "max_in_flight": self.max_active, "slots": len(self.threads), "hbm_budget": self.budget,
                "resident": self.resident, "reused": sum(r.reused for r in self.finished),
                "mean_batch": float(np.mean([r.batch for r in self.finished]))}
