"""ctypes binding of libbddc.so (argument marshalling only).

Every step of the method runs in the library's HIP kernels; this module only
converts Python objects into the C structures of include/bddc.h, passes device
pointers of torch tensors through, and turns status codes into exceptions.
It fails loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbddc.so")
MAX_LEVELS = 8

STATUS = {0: "BDDC_OK", -1: "BDDC_EINVAL", -2: "BDDC_ENOMEM", -3: "BDDC_ESINGULAR",
          -4: "BDDC_EPARTITION", -5: "BDDC_ENOCONV", -6: "BDDC_EDEVICE", -7: "BDDC_EBUSY",
          -8: "BDDC_EUNSUPPORTED"}
ELEMENT = {"Q1": 0, "P1": 1, "Q1E": 2}   # Q1E: plane elasticity, two dofs per node
CONSTRAINTS = {"corners": 0, "corners_edges": 1, "adaptive": 2}
PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2}


class BddcProblemC(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("element", ctypes.c_int32),
                ("coeff", ctypes.POINTER(ctypes.c_double)), ("part", ctypes.POINTER(ctypes.c_int32)),
                ("nsub", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("agglom", ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))),
                ("constraints", ctypes.c_int32), ("tau", ctypes.c_double), ("precision", ctypes.c_int32),
                ("coeff_device", ctypes.c_void_p)]


class BddcInfoC(ctypes.Structure):
    _fields_ = [("n_free", ctypes.c_int64), ("levels", ctypes.c_int32),
                ("nsub", ctypes.c_int32 * MAX_LEVELS), ("n_dof", ctypes.c_int32 * MAX_LEVELS),
                ("n_interface", ctypes.c_int32 * MAX_LEVELS), ("n_corners", ctypes.c_int32 * MAX_LEVELS),
                ("n_edges", ctypes.c_int32 * MAX_LEVELS), ("nc", ctypes.c_int32 * MAX_LEVELS),
                ("n_adaptive", ctypes.c_int32 * MAX_LEVELS), ("omega", ctypes.c_double * MAX_LEVELS),
                ("indicator", ctypes.c_double), ("kappa", ctypes.c_double), ("last_iters", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("apply_bytes", ctypes.c_int64),
                ("matvec_bytes", ctypes.c_int64)]


class BddcTuningC(ctypes.Structure):
    _fields_ = [("deep_path", ctypes.c_int32), ("finalize", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("check", ctypes.c_int32), ("available", ctypes.c_int32), ("solve_ms", ctypes.c_double)]


DEEP_PATHS = ("coop", "wide", "fused", "levels")

SYMBOLS = ["bddc_plan", "bddc_setup", "bddc_apply", "bddc_solve", "bddc_solve_noalloc", "bddc_solve_begin",
           "bddc_solve_advance", "bddc_solve_poll", "bddc_solve_end", "bddc_query", "bddc_edge_eigs",
           "bddc_edge_constraints", "bddc_corners", "bddc_timing_start", "bddc_timing_stop", "bddc_get_tuning",
           "bddc_set_tuning", "bddc_autotune", "bddc_last_error", "bddc_status_string", "bddc_destroy"]

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_0911_5730_amd.build`")
    # torch ships its own HIP runtime with the same soname; loading torch first
    # makes the library bind to it, so the process holds a single HIP runtime
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    i32, i64, dbl, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.bddc_plan.argtypes = [P(BddcProblemC), P(BddcInfoC)]
    lib.bddc_setup.argtypes = [P(BddcProblemC), vp, P(vp)]
    lib.bddc_apply.argtypes = [vp, vp, vp, i32, i64, vp]
    lib.bddc_solve.argtypes = [vp, vp, vp, i32, i64, dbl, i32, P(i32), P(dbl), vp]
    lib.bddc_solve_noalloc.argtypes = [vp, vp, vp, i32, i64, dbl, i32, P(i32), P(dbl), vp]
    lib.bddc_solve_begin.argtypes = [vp, vp, i32, i64, dbl, i32, vp]
    lib.bddc_solve_advance.argtypes = [vp, i32]
    lib.bddc_solve_poll.argtypes = [vp, P(i32)]
    lib.bddc_solve_end.argtypes = [vp, vp, i64, P(i32), P(dbl)]
    lib.bddc_query.argtypes = [vp, P(BddcInfoC)]
    lib.bddc_edge_eigs.argtypes = [vp, i32, i32, P(dbl), i32, P(i32), P(i32), P(i32), P(i32)]
    lib.bddc_edge_constraints.argtypes = [vp, i32, i32, P(i32), i32, P(dbl), i32, P(i32), P(i32)]
    lib.bddc_corners.argtypes = [vp, i32, P(i32), i32, P(i32)]
    lib.bddc_timing_start.argtypes = [ctypes.c_char_p, i32]
    lib.bddc_timing_stop.argtypes = [P(dbl), P(i64), P(dbl), P(dbl)]
    lib.bddc_get_tuning.argtypes = [vp, P(BddcTuningC)]
    lib.bddc_set_tuning.argtypes = [vp, P(BddcTuningC)]
    lib.bddc_autotune.argtypes = [vp, vp, vp, i32, i64, dbl, i32, P(BddcTuningC), vp]
    lib.bddc_status_string.argtypes = [i32]
    lib.bddc_status_string.restype = ctypes.c_char_p
    lib.bddc_destroy.argtypes = [vp]
    lib.bddc_destroy.restype = None
    lib.bddc_last_error.argtypes = []
    lib.bddc_last_error.restype = ctypes.c_char_p
    for name in SYMBOLS[:-3]:
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


class BDDCError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        detail = ""
        if _lib is not None:
            detail = (_lib.bddc_last_error() or b"").decode(errors="replace")
        super().__init__(f"{where}: {self.name}" + (f" ({detail})" if detail else ""))


def _check(st: int, where: str):
    if st != 0:
        raise BDDCError(st, where)


class _Marshalled:
    """C view of a problem; keeps the numpy buffers alive while in use."""

    def __init__(self, prob, tau=None, constraints=None, precision="fp64", coeff_device=None):
        self.coeff = np.ascontiguousarray(prob.coeff, dtype=np.float64)
        self.part = np.ascontiguousarray(prob.part, dtype=np.int32)
        self.agg = [np.ascontiguousarray(a, dtype=np.int32) for a in (prob.agglom or [])]
        ne = int(prob.nx) * int(prob.ny)
        if prob.nx >= 2 and prob.ny >= 2 and (self.coeff.size != ne or self.part.size != ne):
            raise ValueError("coeff and part must have nx*ny entries")
        nprev = prob.nsub
        for a in self.agg:
            if a.size != nprev:
                raise ValueError("each agglomeration array needs one entry per substructure")
            nprev = int(a.max()) + 1 if a.size else 0
        n = max(1, len(self.agg))
        self.agg_ptrs = (ctypes.POINTER(ctypes.c_int32) * n)()
        for i, a in enumerate(self.agg):
            self.agg_ptrs[i] = a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        kind = constraints or prob.constraints
        t = prob.tau if tau is None else tau
        self.c = BddcProblemC(
            nx=prob.nx, ny=prob.ny, element=ELEMENT[prob.element],
            coeff=self.coeff.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            part=self.part.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            nsub=prob.nsub, levels=prob.levels,
            agglom=ctypes.cast(self.agg_ptrs, ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)))
            if self.agg else None,
            constraints=CONSTRAINTS[kind], tau=float(t) if math.isfinite(t) else float("inf"),
            precision=PRECISION[precision] if isinstance(precision, str) else int(precision))
        if coeff_device is not None:
            self.c.coeff_device = ctypes.c_void_p(coeff_device)


def info_dict(ci: BddcInfoC) -> dict:
    L = max(1, ci.levels - 1)
    per = lambda arr: [arr[i] for i in range(L)]
    return dict(n_free=ci.n_free, levels=ci.levels, nsub=per(ci.nsub), n_dof=per(ci.n_dof),
                n_interface=per(ci.n_interface), n_corners=per(ci.n_corners), n_edges=per(ci.n_edges),
                nc=per(ci.nc), n_adaptive=per(ci.n_adaptive), omega=per(ci.omega),
                indicator=ci.indicator, kappa=ci.kappa, last_iters=ci.last_iters,
                device_bytes=ci.device_bytes, apply_bytes=ci.apply_bytes, matvec_bytes=ci.matvec_bytes)


def plan(prob, **kw) -> dict:
    """Host-only validation and level-1 topology (bddc_plan)."""
    lib = load_library()
    m = _Marshalled(prob, **kw)
    ci = BddcInfoC()
    _check(lib.bddc_plan(ctypes.byref(m.c), ctypes.byref(ci)), "bddc_plan")
    d = info_dict(ci)
    return {k: (v[0] if isinstance(v, list) else v) for k, v in d.items()}


def footprint(prob) -> int:
    """Device bytes a set-up of the problem will hold (bddc_plan, no device work)."""
    return int(plan(prob)["device_bytes"])


def _stream_ptr(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _vec_args(t, n_free):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    if t.dim() == 1:
        if t.shape[0] != n_free:
            raise ValueError("vector length must be n_free")
        return 1, n_free
    if t.dim() == 2 and t.shape[1] == n_free:
        return t.shape[0], n_free
    raise ValueError("expected shape (n_free,) or (nrhs, n_free)")


class Solver:
    """A set-up adaptive-multilevel BDDC preconditioner on the current GPU."""

    def __init__(self, prob, *, tau=None, constraints=None, precision="fp64", stream=None, coeff=None):
        """coeff: optional float64 CUDA tensor with the nx*ny coefficients (kept on the device)."""
        self.lib = load_library()
        dptr = None
        if coeff is not None:
            import torch
            if not (coeff.is_cuda and coeff.dtype == torch.float64 and coeff.is_contiguous()
                    and coeff.numel() == prob.nx * prob.ny):
                raise TypeError("coeff must be a contiguous float64 CUDA tensor with nx*ny entries")
            dptr = coeff.data_ptr()
        m = _Marshalled(prob, tau=tau, constraints=constraints, precision=precision, coeff_device=dptr)
        h = ctypes.c_void_p()
        _check(self.lib.bddc_setup(ctypes.byref(m.c), ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(h)),
               "bddc_setup")
        self.h = h
        self.n_free = (2 if prob.element == "Q1E" else 1) * (prob.nx - 1) * (prob.ny - 1)
        self.levels = prob.levels

    def close(self):
        if getattr(self, "h", None):
            self.lib.bddc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def info(self) -> dict:
        ci = BddcInfoC()
        _check(self.lib.bddc_query(self.h, ctypes.byref(ci)), "bddc_query")
        return info_dict(ci)

    def apply(self, r, z=None, stream=None):
        import torch
        nrhs, ld = _vec_args(r, self.n_free)
        if z is None:
            z = torch.empty_like(r)
        _check(self.lib.bddc_apply(self.h, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                   nrhs, ld, ctypes.c_void_p(_stream_ptr(stream))), "bddc_apply")
        return z

    def solve(self, f, u=None, rtol=1e-8, maxit=1000, stream=None, allow_noconv=False):
        import torch
        nrhs, ld = _vec_args(f, self.n_free)
        if u is None:
            u = torch.empty_like(f)
        iters = (ctypes.c_int32 * nrhs)()
        relres = (ctypes.c_double * nrhs)()
        st = self.lib.bddc_solve(self.h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()), nrhs, ld,
                                 float(rtol), int(maxit), iters, relres, ctypes.c_void_p(_stream_ptr(stream)))
        if not (st == -5 and allow_noconv):
            _check(st, "bddc_solve")
        return u, list(iters), list(relres)

    # stepwise solve (bddc_solve_begin / _advance / _poll / _end)
    def begin(self, f, rtol=1e-8, maxit=1000, stream=None):
        nrhs, ld = _vec_args(f, self.n_free)
        self._step_f = f   # kept alive until end()
        _check(self.lib.bddc_solve_begin(self.h, ctypes.c_void_p(f.data_ptr()), nrhs, ld, float(rtol), int(maxit),
                                         ctypes.c_void_p(_stream_ptr(stream))), "bddc_solve_begin")

    def advance(self, iterations=8):
        _check(self.lib.bddc_solve_advance(self.h, int(iterations)), "bddc_solve_advance")

    def poll(self) -> int:
        st = ctypes.c_int32()
        _check(self.lib.bddc_solve_poll(self.h, ctypes.byref(st)), "bddc_solve_poll")
        return st.value

    def end(self, u=None, allow_noconv=False):
        import torch
        f = self._step_f
        nrhs, ld = _vec_args(f, self.n_free)
        if u is None:
            u = torch.empty_like(f)
        iters = (ctypes.c_int32 * nrhs)()
        relres = (ctypes.c_double * nrhs)()
        st = self.lib.bddc_solve_end(self.h, ctypes.c_void_p(u.data_ptr()), ld, iters, relres)
        self._step_f = None
        if not (st == -5 and allow_noconv):
            _check(st, "bddc_solve_end")
        return u, list(iters), list(relres)

    def tuning(self) -> dict:
        """The handle's launch configuration (bddc_get_tuning)."""
        t = BddcTuningC()
        _check(self.lib.bddc_get_tuning(self.h, ctypes.byref(t)), "bddc_get_tuning")
        return _tuning_dict(t)

    def set_tuning(self, **kw):
        """Change knobs of the launch configuration: deep_path ("coop", "wide",
        "fused", "levels"), finalize, graph (0/1), check (4, 8, 16)."""
        t = BddcTuningC()
        _check(self.lib.bddc_get_tuning(self.h, ctypes.byref(t)), "bddc_get_tuning")
        for k, v in kw.items():
            setattr(t, k, DEEP_PATHS.index(v) if k == "deep_path" else int(v))
        _check(self.lib.bddc_set_tuning(self.h, ctypes.byref(t)), "bddc_set_tuning")

    def autotune(self, f, u=None, rtol=1e-8, reps=3, stream=None) -> dict:
        """Time bddc_solve of f under the available launch configurations and
        keep the fastest (bddc_autotune); returns the chosen configuration."""
        import torch
        nrhs, ld = _vec_args(f, self.n_free)
        if u is None:
            u = torch.empty_like(f)
        t = BddcTuningC()
        _check(self.lib.bddc_autotune(self.h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()), nrhs,
                                      ld, float(rtol), int(reps), ctypes.byref(t),
                                      ctypes.c_void_p(_stream_ptr(stream))), "bddc_autotune")
        return _tuning_dict(t)

    def edge_eigs(self, level: int, edge: int):
        n_lam, n_sel, ned = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        pair = (ctypes.c_int32 * 2)()
        _check(self.lib.bddc_edge_eigs(self.h, level, edge, None, 0, ctypes.byref(n_lam), ctypes.byref(n_sel),
                                       pair, ctypes.byref(ned)), "bddc_edge_eigs")
        lam = (ctypes.c_double * max(1, n_lam.value))()
        _check(self.lib.bddc_edge_eigs(self.h, level, edge, lam, n_lam.value, None, None, None, None),
               "bddc_edge_eigs")
        return np.array(lam[:n_lam.value]), n_sel.value, (pair[0], pair[1])

    def edge_constraints(self, level: int, edge: int):
        ne, m = ctypes.c_int32(), ctypes.c_int32()
        _check(self.lib.bddc_edge_constraints(self.h, level, edge, None, 0, None, 0, ctypes.byref(ne),
                                              ctypes.byref(m)), "bddc_edge_constraints")
        dofs = (ctypes.c_int32 * max(1, ne.value))()
        q = (ctypes.c_double * max(1, ne.value * m.value))()
        _check(self.lib.bddc_edge_constraints(self.h, level, edge, dofs, ne.value, q, ne.value * m.value, None,
                                              None), "bddc_edge_constraints")
        Q = np.array(q[:ne.value * m.value]).reshape(m.value, ne.value).T
        return np.array(dofs[:ne.value]), Q


    def corners(self, level: int) -> np.ndarray:
        """Corner dofs of a level, ascending (bddc_corners)."""
        n = ctypes.c_int32()
        _check(self.lib.bddc_corners(self.h, level, None, 0, ctypes.byref(n)), "bddc_corners")
        buf = (ctypes.c_int32 * max(1, n.value))()
        _check(self.lib.bddc_corners(self.h, level, buf, n.value, None), "bddc_corners")
        return np.array(buf[:n.value], dtype=np.int64)


def _tuning_dict(t: BddcTuningC) -> dict:
    return {"deep_path": DEEP_PATHS[t.deep_path], "finalize": t.finalize, "graph": t.graph, "check": t.check,
            "available": [p for i, p in enumerate(DEEP_PATHS) if t.available >> i & 1], "solve_ms": t.solve_ms}


def timing_start(kernel: str, every: int = 1):
    """Arm HIP-event timing on one in `every` launches of one library kernel."""
    _check(load_library().bddc_timing_start(kernel.encode(), int(every)), "bddc_timing_start")


def timing_stop() -> dict:
    """Summed kernel time (ms), launches, algorithmic bytes and flops since timing_start."""
    ms, n, by, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    _check(load_library().bddc_timing_stop(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by),
                                           ctypes.byref(fl)), "bddc_timing_stop")
    return dict(ms=ms.value, launches=n.value, bytes=by.value, flops=fl.value)


def status_string(code: int) -> str:
    return load_library().bddc_status_string(code).decode()


def exported_symbols(path: str = LIB_PATH) -> Sequence[str]:
    lib = ctypes.CDLL(path)
    return [s for s in SYMBOLS if hasattr(lib, s)]
