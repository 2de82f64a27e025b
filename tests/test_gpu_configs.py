"""GPU parity at the workload sizes.

* 256 x 256, 16 x 16 substructures, three levels, adaptive tau = 10 with
  coefficient jumps up to 1e6 and channels: the whole oracle runs (about a
  minute on the host) and every edge's eigenvalues, selection and the solve
  are compared.
* 1024 x 1024, 64 x 64 substructures, three levels, k = 1: too large for the
  oracle's setup, so the checks are properties that hold at any size (true
  residual, symmetry of the preconditioner), the energy-norm error of the
  FP64, FP32 and BF16 solutions against a sparse direct solve of the oracle's
  assembled matrix (at most 1e-8), and the interior-edge pair eigenvalues,
  which for k = 1 coincide with those of the same floating pair in a 4 x 4
  partition that the oracle solves.
* 2048 x 2048, 1024 uneven Voronoi regions of 3000-5700 dofs, eight loads:
  the true residual of every column, the energy-norm error of the FP32 form
  against the FP64 path converged to 1e-12, and a column solved alone
  against the blocked column.
"""

import numpy as np
import pytest
import scipy.sparse.linalg  # noqa: F401

import synth
from gpu_common import check_adaptive_edges, check_solution, cuda_vec, run_pair
from oracle import adaptive, fem
from oracle.bddc import BDDC

pytestmark = pytest.mark.gpu


def test_config2_full_parity():
    prob = synth.config(2)
    print("config2: oracle setup (about a minute)", flush=True)
    S, B, ug, it, rr, o = run_pair(prob)
    try:
        print("config2 iters gpu", it, "oracle", o["iters"], flush=True)
        assert abs(it - o["iters"]) <= 1
        info = S.info()
        check_solution(S, B, ug, o)
        assert info["nc"] == B.nc_per_level()
        check_adaptive_edges(S, B, prob.tau)
        assert abs(info["indicator"] - B.indicator) <= 1e-6 * B.indicator
        assert B.indicator <= prob.tau ** (prob.levels - 1)
    finally:
        S.close()


def test_config3_properties_and_sampled_edges():
    import time

    import scipy.sparse.linalg as spla

    import paper_0911_5730_amd as P
    from oracle import pcg
    prob = synth.config(3)
    A = fem.assemble(prob.nx, prob.ny, prob.coeff)
    t0 = time.perf_counter()
    xs = spla.spsolve(A.tocsc(), prob.f[0], permc_spec="MMD_AT_PLUS_A")
    print(f"config3: sparse direct solve of the assembled matrix {time.perf_counter() - t0:.1f} s", flush=True)
    assert np.linalg.norm(A @ xs - prob.f[0]) <= 1e-12 * np.linalg.norm(prob.f[0])
    # the precision forms: the outer FP64 iteration wins the accuracy back
    f = cuda_vec(prob.f[0])
    for prec in ("fp32", "bf16"):
        with P.Solver(prob, precision=prec) as S:
            u, it, rr = S.solve(f)
            ug = u.cpu().numpy()
        res = np.linalg.norm(A @ ug - prob.f[0]) / np.linalg.norm(prob.f[0])
        err = pcg.energy_error(A, ug, xs)
        print(f"config3 {prec}: iterations {it[0]}, true residual {res:.2e}, energy error {err:.2e}", flush=True)
        assert rr[0] <= 1e-8 and res <= 2e-8
        assert err <= 1e-8, (prec, err)
    print("config3: GPU setup + solve", flush=True)
    with P.Solver(prob) as S:
        u, it, rr = S.solve(f)
        info = S.info()
        ug = u.cpu().numpy()
        res = np.linalg.norm(A @ ug - prob.f[0]) / np.linalg.norm(prob.f[0])
        err = pcg.energy_error(A, ug, xs)
        print("config3 iters", it, "relres", rr, "true", res, "energy error", err, "nc", info["nc"], flush=True)
        assert rr[0] <= 1e-8 and res <= 2e-8
        assert err <= 1e-8
        assert info["indicator"] <= prob.tau ** 2
        # symmetry of the three-level preconditioner
        rng = np.random.default_rng(9)
        r, s = rng.standard_normal((2, prob.n_free))
        a = s @ S.apply(cuda_vec(r)).cpu().numpy()
        b = r @ S.apply(cuda_vec(s)).cpu().numpy()
        assert abs(a - b) <= 1e-11 * max(abs(a), abs(b))
        # interior floating pair vs the oracle on a 4 x 4 partition with H/h = 16
        small = synth.square_problem(64, 4, constraints="adaptive", tau=10.0, kmode="one", seed=1)
        lv = BDDC(small).levels[0]
        lam_o = adaptive.pair_eig_full(lv, 5, 6)[0][:15]
        ns = 64
        for (bi, bj) in [(10, 20), (31, 31), (50, 7)]:
            s_id = bj * ns + bi
            key = (s_id, s_id + 1)
            e = _edge_index(S, key)
            lam_g, nsel, pair = S.edge_eigs(1, e)
            assert tuple(pair) == key
            assert np.allclose(lam_g, lam_o, atol=1e-9 * lam_o[0])
            assert nsel == int(np.sum(lam_o > prob.tau))


def _edge_index(S, key):
    # edges are numbered in increasing (s, t) order; binary search through the ABI
    lo, hi = 0, S.info()["n_edges"][0] - 1
    while lo <= hi:
        mid = (lo + hi) // 2
        pair = S.edge_eigs(1, mid)[2]
        if pair == key:
            return mid
        if pair < key:
            lo = mid + 1
        else:
            hi = mid - 1
    raise KeyError(key)


def test_config4_uneven_substructures_eight_loads():
    """2048 x 2048 (4.2M unknowns), 1024 Voronoi regions of about 3000-5700
    local dofs (interior elimination by the tiled MFMA kernel, interior
    solves by tiled block substitution), 16 Voronoi groups, adaptive
    tau = 10, k = 10^U(0,4), eight loads in one blocked solve in the FP32
    form: every column converges with a true residual of the solve's
    tolerance (checked with the oracle's assembled matrix) and lies within
    1e-8 in the energy norm of the FP64 path converged to 1e-12, and one
    column solved alone gives bitwise the blocked column.  The two forms are
    set up one after the other (each holds about 160 GB of dense local
    matrices)."""
    import time

    import torch

    import paper_0911_5730_amd as P
    from oracle import pcg
    prob = synth.config(4, nrhs=8)
    print(f"config4: {prob.nsub} regions, {prob.n_free} unknowns", flush=True)
    F = cuda_vec(prob.f)
    # reference: the FP64 path (oracle-checked on smaller cases) to 1e-12
    with P.Solver(prob) as S64:
        Uref, itr, rrr = S64.solve(F, rtol=1e-12)
        print(f"config4 FP64 reference iterations {itr}", flush=True)
        assert all(x <= 1e-12 for x in rrr)
        Uref = Uref.cpu().numpy()
    t0 = time.perf_counter()
    S = P.Solver(prob, precision="fp32")
    try:
        torch.cuda.synchronize()
        print(f"config4 setup {time.perf_counter() - t0:.2f} s, nc {S.info()['nc']}", flush=True)
        U, its, rr = S.solve(F)
        print(f"config4 iterations {its}", flush=True)
        assert all(x <= 1e-8 for x in rr)
        u2, it2, _ = S.solve(F[2].contiguous())
        assert it2[0] == its[2] and torch.equal(u2, U[2])
        U = U.cpu().numpy()
    finally:
        S.close()
    A = fem.assemble(prob.nx, prob.ny, prob.coeff)
    for c in range(8):
        nf = np.linalg.norm(prob.f[c])
        res = np.linalg.norm(A @ U[c] - prob.f[c]) / nf
        # the reference reaches the rounding floor of the interface operator
        # (its recursive residual 1e-12; the true one measured about 1e-11)
        res_ref = np.linalg.norm(A @ Uref[c] - prob.f[c]) / nf
        err = pcg.energy_error(A, U[c], Uref[c])
        print(f"config4 column {c}: true residual {res:.2e} (reference {res_ref:.2e}), energy error of the FP32 "
              f"form {err:.2e}", flush=True)
        assert res <= 2e-8, c
        assert res_ref <= 1e-10, c
        assert err <= 1e-8, (c, err)
