"""Blocked right-hand sides: bddc_solve runs up to eight columns in one PCG,
each launch applying its operator block to every column still iterating.

Every column keeps its own recurrences, scalars and convergence test, and
its arithmetic is the single-column arithmetic, so a blocked solve must give
bitwise the iterates of solving each column alone (BDDC_SOLVE_BLOCK=1), for
every deep-level path (with the coarsest problem solved by its Cholesky
factor or by the product with its inverse), precision form and partial-sum
mode (and interfaces
whose column slots do not fill a workgroup: 129-192 dofs), with columns
that converge at different iterations (one at once: a zero load), a ragged
last block (11 columns = 8 + 3), and a changing block width between solves
on one handle (the captured chunk of launches is rebuilt).  The blocked
solutions must also match the FP64 oracle.
"""

import numpy as np
import pytest

from gpu_common import cuda_vec, direct
from oracle import pcg
from oracle.bddc import BDDC
from test_gpu_parity import _case

pytestmark = pytest.mark.gpu


def _loads(prob, k, seed):
    """k load columns: seeded uniform, a smooth one, a scaled copy and a zero
    column, so that the columns finish at different iterations."""
    rng = np.random.default_rng(seed)
    F = rng.uniform(-1.0, 1.0, size=(k, prob.n_free))
    F[0] = prob.f[0]
    if k > 2:
        F[1] = 1.0                      # smooth load: fewer iterations
    if k > 3:
        F[2] = 1e-6 * F[0]              # same direction, scaled
    if k > 4:
        F[3] = 0.0                      # converged before the first iteration
    return F


def _alone(S, F, monkeypatch, **kw):
    import torch
    monkeypatch.setenv("BDDC_SOLVE_BLOCK", "1")
    U, its = [], []
    for c in range(F.shape[0]):
        u, it, _ = S.solve(cuda_vec(F[c]), **kw)
        U.append(u)
        its += it
    monkeypatch.delenv("BDDC_SOLVE_BLOCK")
    return torch.stack(U), its


@pytest.mark.parametrize("case,path", [("adaptive3", "coop"), ("adaptive3", "wide"), ("adaptive3", "fused"),
                                       ("adaptive3", "levels"), ("corners_kjump", "two-level"),
                                       ("voronoi_jitter3", "default"), ("adaptive3", "wide+inverse"),
                                       ("adaptive3", "levels+inverse"), ("corners_kjump", "two-level+inverse")])
def test_blocked_columns_equal_single_columns_bitwise(case, path, monkeypatch):
    import torch

    import paper_0911_5730_amd as P
    deep, _, coarse = path.partition("+")
    if deep not in ("two-level", "default"):
        monkeypatch.setenv("BDDC_DEEP_PATH", deep)
    if coarse:
        monkeypatch.setenv("BDDC_COARSE", coarse)
    prob = _case(case)
    F = _loads(prob, 11, 3)
    print(f"blocked rhs, case {case}, deep path {path}", flush=True)
    with P.Solver(prob) as S:
        U, its, rr = S.solve(cuda_vec(F), rtol=1e-10)
        Ua, itsa = _alone(S, F, monkeypatch, rtol=1e-10)
        assert its == itsa
        assert its[3] == 0 and len(set(its)) >= 2, its
        assert torch.equal(U, Ua)
        # block width changes on the same handle: 3, then 8 columns
        U3, its3, _ = S.solve(cuda_vec(F[:3]), rtol=1e-10)
        assert its3 == its[:3] and torch.equal(U3, U[:3])
        U8, its8, _ = S.solve(cuda_vec(F[3:]), rtol=1e-10)
        assert its8 == its[3:] and torch.equal(U8, U[3:])


@pytest.mark.parametrize("case,ops,prec", [("adaptive3_h16", "full", "fp64"), ("adaptive3_h16", "full", "fp32"),
                                           ("voronoi_jitter3", "packed", "fp32"), ("voronoi_jitter3", "rows", "fp64"),
                                           ("voronoi_jitter3", "rows", "fp32"), ("adaptive3_h16", "rows", "fp32")])
def test_blocked_pcg_operator_storage(case, ops, prec, monkeypatch):
    """S_s and T_rr as packed lower triangles or as full matrices (wide
    interfaces use the full form), and the product and update/restriction by
    64-row blocks with a workgroup per block (the launches of interfaces
    wider than a workgroup; here interfaces of one to three blocks): blocked
    columns bitwise equal to single ones in every form."""
    import torch

    import paper_0911_5730_amd as P
    if ops == "rows":
        monkeypatch.setenv("BDDC_PCG_ROWS", "1")
    else:
        monkeypatch.setenv("BDDC_PCG_OPS", ops)
    prob = _case(case)
    F = _loads(prob, 5, 4)
    print(f"operator storage {ops}, case {case}, {prec}", flush=True)
    with P.Solver(prob, precision=prec) as S:
        U, its, _ = S.solve(cuda_vec(F), rtol=1e-10)
        Ua, itsa = _alone(S, F, monkeypatch, rtol=1e-10)
        assert its == itsa
        assert torch.equal(U, Ua)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("fin", ["0", "1", "2", "3"])
def test_blocked_precision_forms_and_partial_sums(prec, fin, monkeypatch):
    import torch

    import paper_0911_5730_amd as P
    monkeypatch.setenv("BDDC_PCG_FINALIZE", fin)
    prob = _case("adaptive3")
    F = _loads(prob, 6, 4)
    print(f"blocked rhs, precision {prec}, finalize {fin}", flush=True)
    with P.Solver(prob, precision=prec) as S:
        U, its, _ = S.solve(cuda_vec(F))
        Ua, itsa = _alone(S, F, monkeypatch)
        assert its == itsa
        assert torch.equal(U, Ua)


def test_blocked_solutions_match_oracle():
    import paper_0911_5730_amd as P
    prob = _case("adaptive3_h16")
    F = _loads(prob, 8, 5)
    B = BDDC(prob)
    xs = [direct(B, F[c]) for c in (0, 1, 4, 7)]
    with P.Solver(prob) as S:
        U, its, rr = S.solve(cuda_vec(F))
        U = U.cpu().numpy()
    for k, c in enumerate((0, 1, 4, 7)):
        o = pcg.solve(B, F[c], rtol=1e-8)
        assert abs(its[c] - o["iters"]) <= 1, (c, its[c], o["iters"])
        e = pcg.energy_error(B.A, U[c], xs[k])
        e_or = pcg.energy_error(B.A, o["x"], xs[k])
        assert e <= max(1e-10, 2.0 * e_or), (c, e, e_or)
        assert rr[c] <= 1e-8


def test_blocked_maxit_reports_noconv_per_column():
    import paper_0911_5730_amd as P
    prob = _case("corners_kjump")
    F = _loads(prob, 5, 6)
    with P.Solver(prob) as S:
        with pytest.raises(P.BDDCError) as ei:
            S.solve(cuda_vec(F), maxit=3)
        assert ei.value.name == "BDDC_ENOCONV"
        U, its, rr = S.solve(cuda_vec(F), maxit=3, allow_noconv=True)
        assert its == [3, 3, 3, 0, 3]
        assert np.isfinite(U.cpu().numpy()).all()
