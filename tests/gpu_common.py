"""Shared helpers of the GPU parity tests (test infrastructure)."""

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import pcg
from oracle.bddc import BDDC


def cuda_vec(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


TIGHT = 1e-10     # PCG tolerance at which the 1e-10 energy-norm bar is applied
# relative eigenvalue tolerance of the pair eigenproblems: the largest
# eigenvalues (lambda >> tau) are ill-conditioned with respect to the rounding
# of the local matrices (a 1e-16 relative perturbation of K moves lambda_max
# by ~1e-9 at level 1, measured on the oracle), and level-2 matrices carry the
# rounding of the level-1 coarse solves
LAM_RTOL = 1e-6


def run_pair(prob, rtol=1e-8, maxit=1000, oracle=None, tuning=None):
    """Solve the same problem with the GPU library (launch configuration
    `tuning`, if given) and the oracle."""
    import paper_0911_5730_amd as P
    B = oracle or BDDC(prob)
    S = P.Solver(prob)
    if tuning:
        S.set_tuning(**tuning)
    f = cuda_vec(prob.f[0])
    u, it, rr = S.solve(f, rtol=rtol, maxit=maxit)
    o = pcg.solve(B, prob.f[0], rtol=rtol, maxit=maxit)
    return S, B, u.cpu().numpy(), it[0], rr[0], o


def check_solution(S, B, ug, o, rtol=1e-8):
    """Parity of the solutions.

    At the production tolerance the iterates still carry an error of about
    rtol * sqrt(cond) against the exact solution, and rounding-level changes
    of either side move them by about that much (measured on the oracle: a
    1e-15 relative perturbation of its own preconditioner output moves a
    rtol-1e-8 iterate by 1.1e-9, the size of its error).  There the GPU
    iterate's error against the direct solution must be of the oracle's size
    (at most four times it, or 1e-10).  The 1e-10 energy-norm parity bar is
    applied to both sides converged to rtol = 1e-10, with iteration counts
    within +-1."""
    A = B.A
    f = B.prob.f[0]
    r = A @ ug - f
    assert np.linalg.norm(r) <= 2 * rtol * np.linalg.norm(f) + 1e-300
    xs = direct(B)
    e_or = pcg.energy_error(A, o["x"], xs)
    e_g = pcg.energy_error(A, ug, xs)
    assert e_g <= max(1e-10, 4.0 * e_or), f"GPU error {e_g:.3e} vs oracle error {e_or:.3e}"
    ut, it, _ = S.solve(cuda_vec(f), rtol=TIGHT)
    ot = pcg.solve(B, f, rtol=TIGHT)
    assert abs(it[0] - ot["iters"]) <= 1, (it[0], ot["iters"])
    et = pcg.energy_error(A, ut.cpu().numpy(), ot["x"])
    assert et <= 1e-10, f"energy-norm difference at rtol {TIGHT}: {et:.3e}"


def check_adaptive_edges(S, B, tau, levels_to_span=(1,)):
    """Per-edge eigenvalues, selection counts and constraint spans against the oracle."""
    for li, lv in enumerate(B.levels):
        lam_o = B.eigs[li]
        keys = list(lv.topo.edges.keys())
        for e, key in enumerate(keys):
            lam_g, nsel_g, pair = S.edge_eigs(li + 1, e)
            assert tuple(pair) == key
            lo = lam_o[key]
            assert len(lam_g) == len(lo)
            # FP64 roundoff times the pencil's condition (k contrast up to 1e6 times (H/h)^2)
            scale = max(1.0, float(lo[0]))
            tol = LAM_RTOL * np.maximum(1.0, np.abs(lo)) + 1e-10 * scale
            assert np.all(np.abs(lam_g - lo) <= tol), (li, key, lam_g[:4], lo[:4])
            near = np.any(np.abs(lo - tau) <= 1e-8 * max(1.0, tau))
            if not near:
                assert nsel_g == int(np.sum(lo > tau)), (li, key)
            if (li + 1) in levels_to_span and not near:
                dofs, Qg = S.edge_constraints(li + 1, e)
                assert np.array_equal(dofs, lv.topo.edges[key])
                Qo = B.edge_Q[li][key]
                assert Qg.shape[1] == Qo.shape[1]
                if Qo.shape[1]:
                    assert np.allclose(Qg.T @ Qg, np.eye(Qg.shape[1]), atol=1e-10)
                    ang = sla.subspace_angles(Qg, Qo)
                    assert np.max(ang) < 1e-6, (li, key, np.max(ang))


# entrywise bar of the preconditioner apply: |z_gpu - z_oracle| <=
# APPLY_ATOL * max|z_oracle| + APPLY_RTOL * |z_oracle| on every entry.  The
# two sides apply the same operator with different algorithms (explicit
# constrained inverses and dense interior inverses against KKT and sparse LU
# solves), so every entry carries rounding of order eps times the local
# condition numbers (coefficient jumps up to 1e6, H/h up to 32) relative to
# the largest entries of the local solutions
APPLY_ATOL = 1e-11
APPLY_RTOL = 1e-10


def check_apply(zg, zo, atol=APPLY_ATOL, rtol=APPLY_RTOL, tag=""):
    """Entrywise comparison of two preconditioner applies."""
    zg = np.asarray(zg)
    zo = np.asarray(zo)
    assert zg.shape == zo.shape and np.isfinite(zg).all()
    d = np.abs(zg - zo)
    scale = float(np.max(np.abs(zo))) if zo.size else 0.0
    bound = atol * scale + rtol * np.abs(zo)
    worst = int(np.argmax(d - bound)) if zo.size else 0
    print(f"apply {tag}: max |dz|/max|z| = {float(d.max()) / max(scale, 1e-300):.2e}, "
          f"worst entry {worst}: dz {d[worst]:.2e} bound {bound[worst]:.2e}", flush=True)
    assert np.all(d <= bound), (tag, worst, d[worst], bound[worst])


def check_topology(S, B):
    """Corner sets and every edge's dof list, at every level, bit-exact
    against the oracle's classification (level-l dofs for l >= 2 are the
    level-(l-1) coarse dofs, numbered the same way on both sides)."""
    for li, lv in enumerate(B.levels):
        cg = S.corners(li + 1)
        assert np.array_equal(cg, np.asarray(lv.topo.corners, dtype=np.int64)), (li, cg[:8])
        keys = list(lv.topo.edges.keys())
        assert S.info()["n_edges"][li] == len(keys)
        for e, key in enumerate(keys):
            dofs, _ = S.edge_constraints(li + 1, e)
            assert np.array_equal(dofs, lv.topo.edges[key]), (li, key)


def direct(B, b=None):
    return spla.spsolve(B.A.tocsc(), B.prob.f[0] if b is None else b)
