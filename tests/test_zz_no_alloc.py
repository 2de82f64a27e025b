"""bddc_solve_noalloc through the C ABI: the per-column PCG state in the
library's fixed device array instead of the handle's arena.  Its results must
be those of bddc_solve (bitwise: the same kernels in the same order), on two
calls in a row with the second on a smaller problem (the array then still
holds the first call's state), and the handle's own solves must be unchanged
afterwards.  A limit below one column's state is refused before any work."""

import ctypes

import numpy as np
import pytest

import synth
from gpu_common import cuda_vec

pytestmark = pytest.mark.gpu


def _noalloc(S, F, rtol=1e-8, maxit=1000):
    import torch
    nrhs = 1 if F.dim() == 1 else F.shape[0]
    U = torch.full_like(F, float("nan"))
    iters = (ctypes.c_int32 * nrhs)()
    relres = (ctypes.c_double * nrhs)()
    st = S.lib.bddc_solve_noalloc(S.h, ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(U.data_ptr()), nrhs,
                                  S.n_free, float(rtol), int(maxit), iters, relres,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return st, U, list(iters), list(relres)


def test_noalloc_solve_matches_solve_twice_then_smaller(monkeypatch):
    import torch

    import paper_0911_5730_amd as P
    big = synth.square_problem(64, 8, levels=3, groups=(2, 2), constraints="adaptive", tau=2.5,
                               kmode="loguniform", kmax_exp=3, channels=2, nrhs=3, seed=26)
    small = synth.square_problem(32, 4, constraints="corners_edges", kmode="loguniform", kmax_exp=2, seed=22)
    Sb = P.Solver(big)
    Ss = P.Solver(small)
    try:
        Fb = cuda_vec(big.f)
        Fs = cuda_vec(small.f[0])
        print("noalloc: three columns on the 64x64 three-level problem", flush=True)
        st, U1, it1, rr1 = _noalloc(Sb, Fb)
        assert st == 0, P.status_string(st)
        Ub, itb, rrb = Sb.solve(Fb)
        assert it1 == itb and rr1 == rrb
        assert torch.equal(U1, Ub)
        print("noalloc: one column on the 32x32 two-level problem", flush=True)
        st, U2, it2, rr2 = _noalloc(Ss, Fs)
        assert st == 0, P.status_string(st)
        Us, its, rrs = Ss.solve(Fs)
        assert it2 == its and torch.equal(U2, Us)
        # the handle's own layout and captured chunk are untouched
        Ub2, itb2, _ = Sb.solve(Fb)
        assert itb2 == itb and torch.equal(Ub2, Ub)
        # a limit below one column's state is refused with nothing done
        monkeypatch.setenv("BDDC_NOALLOC_LIMIT", "4096")
        st, U3, _, _ = _noalloc(Ss, Fs)
        assert st == -8, P.status_string(st)
        assert torch.isnan(U3).all()
        assert "no-allocation scratch" in P.bddc._lib.bddc_last_error().decode()
    finally:
        Sb.close()
        Ss.close()
