"""Serving loop: independent solve requests admitted onto concurrent slots.

Each slot is a host thread with a HIP stream of its own; a request (mesh,
coefficient field, partition, levels, tau, right-hand sides) is set up, solved
and released on the slot that takes it, so the set-up host work of one request
overlaps the kernels of the others and their kernels share the device.  A
request is admitted when a slot is free and the estimated device footprint of
all admitted requests stays within the HBM budget (at least one request is
always admitted, so none starves).  Requests are served in arrival order.
Every numerical step runs in libbddc (bddc_setup / bddc_solve /
bddc_destroy); this module only schedules the calls.

Results do not depend on what else is in flight: each handle has its own
device state and every reduction has a fixed order, so a request's solution
is bitwise the same alone and in the mix (tested).
"""

from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .bddc import Solver


@dataclass
class Request:
    prob: object                       # synth.Problem-like: nx, ny, coeff, part, nsub, levels, agglom, ...
    rhs: np.ndarray                    # (nrhs, n_free) host array
    rtol: float = 1e-8
    precision: str = "fp64"
    arrival: float = 0.0               # seconds, on the server's clock
    # filled in by the server
    admitted: float = 0.0
    done: float = 0.0
    iterations: List[int] = field(default_factory=list)
    solution: Optional[np.ndarray] = None
    footprint: int = 0
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


class Server:
    """Slots of concurrent set-up + solve; see the module docstring."""

    def __init__(self, slots: int = 2, hbm_budget: Optional[int] = None):
        import torch
        self.torch = torch
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.8 * free)
        self.budget = int(hbm_budget)
        self.cv = threading.Condition()
        self.pending: List[Request] = []
        self.finished: List[Request] = []
        self.in_flight = 0                 # admitted bytes
        self.active = 0                    # admitted requests
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

    def _admissible(self) -> Optional[Request]:
        if not self.pending:
            return None
        req = self.pending[0]
        if self.active == 0 or self.in_flight + req.footprint <= self.budget:
            return req
        return None

    def _slot(self, k: int):
        torch = self.torch
        stream = self.streams[k]
        while True:
            with self.cv:
                while True:
                    req = self._admissible()
                    if req is not None or (self.closing and not self.pending):
                        break
                    self.cv.wait()
                if req is None:
                    return
                self.pending.pop(0)
                self.in_flight += req.footprint
                self.active += 1
                self.max_active = max(self.max_active, self.active)
                req.admitted = self.now()
            try:
                with torch.cuda.stream(stream):
                    # (nrhs, n_free) rows are the columns of the library's n_free x nrhs layout
                    f = torch.tensor(np.ascontiguousarray(req.rhs), dtype=torch.float64, device="cuda")
                    S = Solver(req.prob, precision=req.precision, stream=stream)
                    try:
                        u, it, _ = S.solve(f, rtol=req.rtol, stream=stream)
                        req.solution = u.cpu().numpy()
                        req.iterations = [int(x) for x in it]
                    finally:
                        S.close()
            except BaseException as e:  # reported on the request
                req.error = e
            with self.cv:
                req.done = self.now()
                self.in_flight -= req.footprint
                self.active -= 1
                self.finished.append(req)
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

    def stats(self) -> dict:
        lat = np.array([r.latency for r in self.finished]) * 1e3
        span = max(r.done for r in self.finished) - min(r.arrival for r in self.finished)
        return {"requests": len(self.finished), "solves_per_s": len(self.finished) / span,
                "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                "max_in_flight": self.max_active, "slots": len(self.threads), "hbm_budget": self.budget}
