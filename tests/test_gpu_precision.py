"""Precision forms of the interface preconditioner against the FP64 oracle.

In the FP32 and BF16 forms the level-1 T_rr and Psi that the PCG
preconditioner streams every iteration are stored in reduced precision (the
BF16 form keeps T_rr as a diagonally scaled inverse Cholesky factor in BF16
and an FP32 constraint projector) and multiplied in FP64; the outer PCG
recurrences, residuals and inner products, the interface operator S, the
averaging, the deeper levels and the coarsest factor stay FP64.  The outer
iteration then wins the accuracy back: at rtol = 1e-8 the solution must have
the true residual of the FP64 solve and an energy-norm error against the
direct FP64 solution no larger than the FP64 oracle's own PCG iterate (or
1e-8); converged further (1e-10) the error must fall below 1e-9, i.e. the
reduced storage limits only the convergence rate, not the attainable accuracy.
"""

import numpy as np
import pytest

from gpu_common import cuda_vec, direct
from oracle import pcg
from oracle.bddc import BDDC
from test_gpu_parity import _case

pytestmark = pytest.mark.gpu

PREC_CASES = ["config1", "corners_kjump", "adaptive3", "adaptive3_h16"]


@pytest.mark.parametrize("name", PREC_CASES)
def test_precision_forms_reach_fp64_accuracy(name):
    import paper_0911_5730_amd as P

    prob = _case(name)
    B = BDDC(prob)
    A = B.A
    f = prob.f[0]
    xs = direct(B)
    o = pcg.solve(B, f, rtol=1e-8)
    e_or = pcg.energy_error(A, o["x"], xs)
    S64 = P.Solver(prob)
    try:
        _, it64, _ = S64.solve(cuda_vec(f), rtol=1e-8)
    finally:
        S64.close()
    for prec in ("fp32", "bf16"):
        print(f"case {name} precision {prec}", flush=True)
        S = P.Solver(prob, precision=prec)
        try:
            u, it, rr = S.solve(cuda_vec(f), rtol=1e-8)
            ug = u.cpu().numpy()
            assert rr[0] <= 1e-8
            r = A @ ug - f
            assert np.linalg.norm(r) <= 2e-8 * np.linalg.norm(f)
            e = pcg.energy_error(A, ug, xs)
            ut, itt, _ = S.solve(cuda_vec(f), rtol=1e-10)
            et = pcg.energy_error(A, ut.cpu().numpy(), xs)
            print(f"  iterations {it[0]} (FP64 {it64[0]}, oracle {o['iters']}), energy error {e:.2e} "
                  f"(oracle {e_or:.2e}); at 1e-10: {itt[0]} iterations, error {et:.2e}", flush=True)
            assert e <= max(1e-8, 4.0 * e_or), (prec, e, e_or)
            assert et <= 1e-9, (prec, et)
            assert it[0] <= 2 * it64[0] + 5, (prec, it[0], it64[0])
        finally:
            S.close()
