"""Pins of the oracle's BDDC against what the paper and the mathematics fix.

Each test checks the oracle against a definition it does not use itself:
an explicit basis of W-tilde, brute-force eigenproblems, exactness cases,
symmetry and invariance properties (no GPU).
"""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import synth
from oracle import adaptive, pcg
from oracle.bddc import BDDC


def tiny(kind="corners", nx=12, ns=3, levels=2, groups=(1, 1), tau=float("inf"), seed=7,
         kmax=2.0, channels=0, element="Q1"):
    return synth.square_problem(nx, ns, levels=levels, groups=groups, constraints=kind, tau=tau,
                                kmode="loguniform", kmax_exp=kmax, channels=channels, seed=seed,
                                element=element)


# ---------------------------------------------------------------- helpers
def _agreement_rows(lv, positions_of):
    """Rows stating that every coarse functional has one common value across its
    owner substructures, on a concatenated vector of per-substructure blocks."""
    owners = [[] for _ in range(lv.Nc)]
    for s in range(lv.nsub):
        for r, k in enumerate(lv.cids[s]):
            owners[k].append((s, r))
    rows = []
    for k, ow in enumerate(owners):
        s0, r0 = ow[0]
        for s1, r1 in ow[1:]:
            row = np.zeros(positions_of["total"])
            row[positions_of[s0]] += lv.C[s0][r0][positions_of["cols", s0]]
            row[positions_of[s1]] -= lv.C[s1][r1][positions_of["cols", s1]]
            rows.append(row)
    return np.array(rows)


def _full_layout(lv):
    pos, off = {}, 0
    for s in range(lv.nsub):
        n = len(lv.topo.local[s])
        pos[s] = np.arange(off, off + n)
        pos["cols", s] = np.arange(n)
        off += n
    pos["total"] = off
    return pos


def _gamma_layout(lv):
    pos, off = {}, 0
    for s in range(lv.nsub):
        g = lv.interface_positions(s)
        pos[s] = np.arange(off, off + len(g))
        pos["cols", s] = g
        off += len(g)
    pos["total"] = off
    return pos


def _brute_omega(lv):
    """omega = sup over discrete harmonic w in W-tilde of |(I-E)w|_S^2 / |w|_S^2
    (Lemma of Section 2.1), from an explicit basis of W-tilde on the interface."""
    pos = _gamma_layout(lv)
    V = sla.null_space(_agreement_rows(lv, pos)) if lv.Nc else np.eye(pos["total"])
    S = sla.block_diag(*[lv.schur(s) for s in range(lv.nsub)])
    n = pos["total"]
    Emat = np.zeros((n, n))
    # (E w) copied back to every copy: sum_j delta_j(x) w_j(x)
    where = {}
    for s in range(lv.nsub):
        for p, col in zip(pos[s], pos["cols", s]):
            d = int(lv.topo.local[s][col])
            where.setdefault(d, []).append((p, lv.delta[s][col]))
    for d, lst in where.items():
        for p, _ in lst:
            for q, w in lst:
                Emat[p, q] += w
    IE = np.eye(n) - Emat
    X = V.T @ IE.T @ S @ IE @ V
    Y = V.T @ S @ V
    lam = sla.eigh(0.5 * (X + X.T), 0.5 * (Y + Y.T), eigvals_only=True)
    return lam[-1]


def _dense_MA_eigs(B):
    Minv = B.dense_preconditioner()
    A = B.A.toarray()
    assert np.allclose(Minv, Minv.T, atol=1e-12 * np.abs(Minv).max())
    Mmat = np.linalg.inv(0.5 * (Minv + Minv.T))
    return sla.eigh(A, 0.5 * (Mmat + Mmat.T), eigvals_only=True)


# ---------------------------------------------------------------- weights, coarse basis
def test_weights_partition_of_unity_and_equal_split():
    p = tiny("corners_edges")
    lv = BDDC(p).levels[0]
    tot = np.zeros(lv.n)
    for s in range(lv.nsub):
        np.add.at(tot, lv.topo.local[s], lv.delta[s])
    assert np.allclose(tot, 1.0, atol=1e-14)            # E R = I
    q = synth.square_problem(12, 3, kmode="one")
    lv1 = BDDC(q).levels[0]
    for s in range(lv1.nsub):
        for d, w in zip(lv1.topo.local[s], lv1.delta[s]):
            m = len(lv1.topo.N[d])
            assert np.isclose(w, 1.0 / m)                  # k = 1: 1/2 on edges, 1/4 at crosses


@pytest.mark.parametrize("kind", ["corners", "corners_edges"])
def test_coarse_basis_constraints_energy_and_lagrange(kind):
    B = BDDC(tiny(kind))
    lv = B.levels[0]
    for s in range(lv.nsub):
        K, C, Psi = lv.K[s], lv.C[s], lv.Psi[s]
        nc = C.shape[0]
        assert np.allclose(C @ Psi, np.eye(nc), atol=1e-11)
        # energy minimal <=> K-orthogonal to null(C)
        Nul = sla.null_space(C)
        assert np.abs(Nul.T @ K @ Psi).max() < 1e-9 * np.abs(K).max()
        # A_c = -Lambda from the same KKT system
        n = K.shape[0]
        rhs = np.zeros((n + nc, nc))
        rhs[n:] = np.eye(nc)
        Lam = sla.lu_solve(lv.kkt[s], rhs)[n:]
        assert np.allclose(lv.Ac[s], -Lam, atol=1e-9 * np.abs(lv.Ac[s]).max())


def test_a_orthogonal_splitting_of_w_tilde():
    """eq. (tilde-dec): the minimiser over W-tilde of 1/2 a(w,w) - <r_B, E w> is
    w_Delta + w_Pi, and a(w_Delta, w_Pi) = 0."""
    B = BDDC(tiny("corners_edges"))
    lv = B.levels[0]
    rng = np.random.default_rng(1)
    rB = rng.standard_normal(lv.n)
    pos = _full_layout(lv)
    V = sla.null_space(_agreement_rows(lv, pos))
    Kbig = sla.block_diag(*lv.K)
    g = np.concatenate([lv.delta[s] * rB[lv.topo.local[s]] for s in range(lv.nsub)])
    y = np.linalg.solve(V.T @ Kbig @ V, V.T @ g)
    w = V @ y
    gs = [lv.delta[s] * rB[lv.topo.local[s]] for s in range(lv.nsub)]
    wD = np.concatenate([lv.local_solve(s, gs[s]) for s in range(lv.nsub)])
    rc = np.zeros(lv.Nc)
    for s in range(lv.nsub):
        np.add.at(rc, lv.cids[s], lv.Psi[s].T @ gs[s])
    uc = np.linalg.solve(B.A_coarsest, rc)
    wP = np.concatenate([lv.Psi[s] @ uc[lv.cids[s]] for s in range(lv.nsub)])
    assert np.linalg.norm(w - (wD + wP)) <= 1e-11 * np.linalg.norm(w)
    assert abs(wD @ Kbig @ wP) <= 1e-11 * np.sqrt((wD @ Kbig @ wD) * (wP @ Kbig @ wP))


# ---------------------------------------------------------------- spectrum (Lemma)
@pytest.mark.parametrize("kind", ["corners", "corners_edges"])
def test_two_level_spectrum_bounds(kind):
    """lambda_min(M^-1 A) >= 1 and, for two levels, lambda_max = omega exactly
    (E is a projection, so |E| = |I - E| in the energy norm)."""
    B = BDDC(tiny(kind))
    ev = _dense_MA_eigs(B)
    assert ev[0] >= 1.0 - 1e-10
    om = _brute_omega(B.levels[0])
    assert om >= 1.0 - 1e-10
    assert abs(ev[-1] - om) <= 1e-8 * om


def test_three_level_spectrum_bounded_by_product():
    p = tiny("corners", nx=16, ns=4, levels=3, groups=(2, 2))
    B = BDDC(p)
    ev = _dense_MA_eigs(B)
    assert ev[0] >= 1.0 - 1e-10
    om = [_brute_omega(lv) for lv in B.levels]
    assert len(om) == 2 and min(om) >= 1.0 - 1e-10
    assert ev[-1] <= np.prod(om) * (1 + 1e-10)
    # the extra level costs condition number (Tables 1-2 trend)
    B2 = BDDC(p, levels=2)
    assert _dense_MA_eigs(B2)[-1] < ev[-1]


# ---------------------------------------------------------------- exactness
def test_all_interface_coarse_is_exact():
    p = tiny("corners")
    B = BDDC(p, all_interface_corners=True)
    Minv = B.dense_preconditioner()
    Ainv = np.linalg.inv(B.A.toarray())
    assert np.abs(Minv - Ainv).max() <= 1e-11 * np.abs(Ainv).max()
    out = pcg.solve(B, p.f[0], rtol=1e-10)
    assert out["iters"] <= 1


def test_single_level2_substructure_equals_two_level():
    p = tiny("corners", nx=16, ns=4, levels=3, groups=(1, 1))
    M3 = BDDC(p).dense_preconditioner()
    M2 = BDDC(p, levels=2).dense_preconditioner()
    assert np.abs(M3 - M2).max() <= 1e-11 * np.abs(M2).max()


def test_tau_below_every_pair_eigenvalue_is_exact():
    p = tiny("adaptive", tau=1e-6)
    B = BDDC(p)
    lv = B.levels[0]
    for (s, t), E in lv.topo.edges.items():
        assert sum(1 for k in lv.cids[s] if len(lv.func[k][0]) == len(E)
                   and np.array_equal(lv.func[k][0], E)) == len(E)
    out = pcg.solve(B, p.f[0], rtol=1e-10)
    assert out["iters"] <= 1


# ---------------------------------------------------------------- symmetry, invariance
def test_preconditioner_symmetry():
    p = tiny("adaptive", nx=16, ns=4, levels=3, groups=(2, 2), tau=2.0, channels=1)
    B = BDDC(p)
    rng = np.random.default_rng(2)
    r, s = rng.standard_normal((2, B.A.shape[0]))
    a, b = r @ B.apply(s), s @ B.apply(r)
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def test_edge_constraint_basis_invariance():
    p = tiny("adaptive", tau=1.5)
    B = BDDC(p)
    lv = B.levels[0]
    rng = np.random.default_rng(4)
    r = rng.standard_normal(lv.n)
    z0 = B.apply(r)
    # recombine every edge's constraint columns by a random invertible matrix
    newQ = {}
    for key, E in lv.topo.edges.items():
        cols = [lv.func[k][1] for k in range(lv.Nc) if lv.func[k][0] is not None
                and len(lv.func[k][0]) == len(E) and np.array_equal(lv.func[k][0], E)]
        Q = np.array(cols).T.reshape(len(E), len(cols))
        R = rng.standard_normal((Q.shape[1], Q.shape[1])) + 3 * np.eye(Q.shape[1])
        newQ[key] = Q @ R
    assert sum(q.shape[1] for q in newQ.values()) > 0
    lv.build_coarse("adaptive", newQ)
    Ac = np.zeros((lv.Nc, lv.Nc))
    for s in range(lv.nsub):
        Ac[np.ix_(lv.cids[s], lv.cids[s])] += lv.Ac[s]
    B.A_coarsest = Ac
    B.coarse_chol = sla.cho_factor(Ac)
    z1 = B.apply(r)
    assert np.linalg.norm(z1 - z0) <= 1e-10 * np.linalg.norm(z0)


# ---------------------------------------------------------------- PCG, IR form, kappa
def test_fs_and_interface_reduced_iterates_agree():
    """Section 5: reducing level 1 to the interfaces.  An explicit Schur
    complement PCG and the full-space PCG from the condensed start give the
    same interface iterates."""
    p = tiny("corners_edges")
    B = BDDC(p)
    lv = B.levels[0]
    A = B.A.tocsc()
    b = p.f[0]
    I = lv.int_dofs
    G = np.nonzero(~lv.topo.interior)[0]
    AII = spla.splu(A[I][:, I].tocsc())
    AIG = A[I][:, G]
    AGG = A[G][:, G]
    AGI = A[G][:, I]

    def S_apply(x):
        return AGG @ x - AGI @ AII.solve(AIG @ x)

    def M_gamma(r):
        full = np.zeros(lv.n)
        full[G] = r
        return B.apply(full)[G]

    bG = b[G] - AGI @ AII.solve(b[I])
    bnorm_full = np.linalg.norm(b)
    outS = pcg.pcg(S_apply, M_gamma, bG, rtol=1e-8 * bnorm_full / np.linalg.norm(bG),
                   keep_iterates=True)
    outF = pcg.solve(B, b, keep_iterates=True)
    assert outS["iters"] == outF["iters"]
    for xs, xf in zip(outS["iterates"], outF["iterates"]):
        assert np.linalg.norm(xs - xf[G]) <= 1e-11 * np.linalg.norm(xf[G])


def test_pcg_converges_to_direct_solution_and_kappa_estimate():
    p = tiny("corners_edges", nx=16, ns=4)
    B = BDDC(p)
    b = p.f[0]
    out = pcg.solve(B, b, rtol=1e-12)
    xs = spla.spsolve(B.A.tocsc(), b)
    assert pcg.energy_error(B.A, out["x"], xs) < 1e-10
    ev = _dense_MA_eigs(B)
    assert abs(out["kappa"] - ev[-1] / ev[0]) <= 0.01 * ev[-1] / ev[0]


def test_lanczos_tridiagonal_matches_dense_cg_spectrum():
    # plain CG on a diagonal matrix to convergence: the Ritz values are the eigenvalues
    d = np.array([1.0, 2.0, 5.0, 11.0])
    out = pcg.pcg(lambda v: d * v, lambda v: v, np.ones(4), rtol=1e-14)
    T = pcg.lanczos_tridiagonal(out["alphas"], out["betas"])
    assert np.allclose(np.sort(np.linalg.eigvalsh(T)), d, rtol=1e-10)


# ---------------------------------------------------------------- pair eigenproblems
def _pair_cases():
    return [tiny("adaptive", tau=2.0, channels=1, seed=11),
            tiny("adaptive", nx=16, ns=4, levels=3, groups=(2, 2), tau=2.0, channels=1, seed=3)]


def _definition_eigs(lv, s, t):
    """Stationary values of J^st by definition: explicit basis of the pair space
    (shared corners equal), generalized eigenproblem on the complement of the
    zero-energy functions."""
    lam, V, X, info = adaptive.pair_eig_full(lv, s, t)
    n = info["n"]
    gs = lv.interface_positions(s)
    S = sla.block_diag(lv.schur(s), lv.schur(t))
    ps, pt = info["ps"], info["pt"]
    cset = set(int(c) for c in lv.topo.corners)
    rows = []
    IE = np.zeros((n, n))
    for d in info["F"]:
        i, j = ps[int(d)], pt[int(d)]
        a, b = lv.K[s][gs[i], gs[i]], lv.K[t][lv.interface_positions(t)[j - len(gs)],
                                                lv.interface_positions(t)[j - len(gs)]]
        IE[i, [i, j]] = np.array([1, -1]) * b / (a + b)
        IE[j, [j, i]] = np.array([1, -1]) * a / (a + b)
        if int(d) in cset:
            r = np.zeros(n)
            r[i], r[j] = 1, -1
            rows.append(r)
    V0 = sla.null_space(np.array(rows)) if rows else np.eye(n)
    Sv = V0.T @ S @ V0
    w, U = np.linalg.eigh(0.5 * (Sv + Sv.T))
    keep = w > 1e-10 * w.max()
    Wb = V0 @ U[:, keep]
    Xr = Wb.T @ IE.T @ S @ IE @ Wb
    Yr = Wb.T @ S @ Wb
    return np.sort(sla.eigh(0.5 * (Xr + Xr.T), 0.5 * (Yr + Yr.T), eigvals_only=True))[::-1]


@pytest.mark.parametrize("case", [0, 1])
def test_pair_eigen_full_reduced_and_definition_agree(case):
    p = _pair_cases()[case]
    B = BDDC(p)
    for lv in B.levels:
        for (s, t), E in lv.topo.edges.items():
            lam = adaptive.pair_eig_full(lv, s, t)[0][:len(E)]
            red = adaptive.pair_eig_reduced(lv, s, t)[:len(E)]
            dfn = _definition_eigs(lv, s, t)[:len(E)]
            scale = max(1.0, lam[0])
            assert np.allclose(lam, red, atol=1e-10 * scale)
            assert np.allclose(lam, dfn, atol=1e-9 * scale)


def test_constraint_blocks_are_torn_and_augmentation_theorem():
    p = _pair_cases()[0]
    B = BDDC(p)
    lv = B.levels[0]
    checked = 0
    for (s, t), E in lv.topo.edges.items():
        lam, V, X, info = adaptive.pair_eig_full(lv, s, t)
        ps, pt = info["ps"], info["pt"]
        for k in range(len(E)):
            c = X @ V[:, k]
            cs = c[[ps[int(d)] for d in info["F"]]]
            ct = c[[pt[int(d)] for d in info["F"]]]
            assert np.allclose(cs, -ct, atol=1e-10 * np.abs(c).max())      # c^s = -c^t
        for nsel in (1, 2, 3):
            if nsel >= len(E):
                continue
            rows = [X @ V[:, k] for k in range(nsel)]
            rows = [r[[ps[int(d)] for d in E]] for r in rows]
            lam2 = adaptive.pair_eig_full(lv, s, t, extra_rows=rows)[0]
            assert abs(lam2[0] - lam[nsel]) <= 1e-8 * lam[nsel]
            checked += 1
    assert checked > 0


def test_adaptive_setup_meets_target():
    """Theorem "adaptive": after selection every pair's largest remaining
    eigenvalue is <= tau, so omega-tilde <= tau^(L-1); and the preconditioned
    condition number respects the multilevel bound of the Lemma."""
    tau = 2.0
    p = tiny("adaptive", nx=16, ns=4, levels=3, groups=(2, 2), tau=tau, channels=1, seed=3)
    B = BDDC(p)
    assert all(w <= tau for w in B.omega_levels)
    assert B.indicator <= tau ** (p.levels - 1)
    # the coarse dofs actually installed on each edge bring the pair bound down
    # to tau, and the level's omega is the largest pair bound left once every
    # edge carries its installed constraints (Theorem "adaptive": the largest
    # eigenvalue of the augmented pair problem is the first unselected one),
    # computed here from the augmented pencils, not from the selection's lists
    added = 0
    for li, lv in enumerate(B.levels):
        om_aug = 0.0
        for (s, t), E in lv.topo.edges.items():
            rows = [w for d, w in lv.func if len(d) == len(E) and np.array_equal(d, E)]
            lam0 = adaptive.pair_eig_full(lv, s, t)[0][:len(E)]
            assert len(rows) == int(np.sum(lam0 > tau))
            added += len(rows)
            lam1 = adaptive.pair_eig_full(lv, s, t, extra_rows=rows)[0]
            assert lam1[0] <= tau * (1 + 1e-9)
            om_aug = max(om_aug, float(lam1[0]))
        assert abs(B.omega_levels[li] - om_aug) <= 1e-8 * max(1.0, om_aug), (li, B.omega_levels[li], om_aug)
    assert added > 0
    assert abs(B.indicator - np.prod(B.omega_levels)) <= 1e-14 * B.indicator
    ev = _dense_MA_eigs(B)
    om = [_brute_omega(lv) for lv in B.levels]
    assert ev[-1] <= np.prod(om) * (1 + 1e-10)
    # lowering tau adds coarse dofs and lowers the condition number (Tables 6-7)
    Bhi = BDDC(p, tau=20.0)
    assert Bhi.levels[0].Nc <= B.levels[0].Nc
    assert _dense_MA_eigs(Bhi)[-1] >= ev[-1] - 1e-9


def test_p1_elements_run_through_bddc():
    p = tiny("corners_edges", element="P1")
    B = BDDC(p)
    ev = _dense_MA_eigs(B)
    assert ev[0] >= 1 - 1e-10
    assert abs(ev[-1] - _brute_omega(B.levels[0])) <= 1e-8 * ev[-1]


@pytest.mark.parametrize("seed", [41, 42])
def test_voronoi_partition_spectrum_and_adaptive_target(seed):
    """Uneven substructures (Voronoi regions, promoted corners where a pair
    shares none): lambda_min(M^-1 A) >= 1, two-level lambda_max = omega, and
    the adaptive selection brings every pair bound down to tau."""
    p = synth.voronoi_problem(16, 6, constraints="corners", kmode="loguniform", kmax_exp=2.0, seed=seed)
    B = BDDC(p)
    ev = _dense_MA_eigs(B)
    assert ev[0] >= 1.0 - 1e-10
    om = _brute_omega(B.levels[0])
    assert abs(ev[-1] - om) <= 1e-8 * om
    tau = 1.5
    pa = synth.voronoi_problem(16, 6, constraints="adaptive", tau=tau, kmode="loguniform", kmax_exp=2.0,
                               seed=seed)
    Ba = BDDC(pa)
    assert all(w <= tau * (1 + 1e-9) for w in Ba.omega_levels)
    eva = _dense_MA_eigs(Ba)
    assert eva[0] >= 1.0 - 1e-10
    assert eva[-1] <= _brute_omega(Ba.levels[0]) * (1 + 1e-8)
    assert eva[-1] <= ev[-1] + 1e-9


# ---------------------------------------------------------------- elasticity (NEXT-4)
def test_elasticity_two_level_spectrum_bounds_and_direct_solution():
    """Plane-strain elasticity (two dofs per node, the paper's experiment): the
    same Lemma holds -- lambda_min(M^-1 A) >= 1 and lambda_max = omega for two
    levels -- corners carry both components, so a floating substructure's
    three rigid modes are constrained; PCG reaches the direct solution."""
    p = tiny("corners", element="Q1E")
    B = BDDC(p)
    assert B.A.shape[0] == 2 * (p.nx - 1) * (p.ny - 1) == p.n_free
    ev = _dense_MA_eigs(B)
    assert ev[0] >= 1.0 - 1e-10
    om = _brute_omega(B.levels[0])
    assert abs(ev[-1] - om) <= 1e-8 * om
    out = pcg.solve(B, p.f[0], rtol=1e-12)
    xs = spla.spsolve(B.A.tocsc(), p.f[0])
    assert pcg.energy_error(B.A, out["x"], xs) < 1e-10


def test_elasticity_exact_cases():
    p = tiny("corners", element="Q1E")
    B = BDDC(p, all_interface_corners=True)
    Minv = B.dense_preconditioner()
    Ainv = np.linalg.inv(B.A.toarray())
    assert np.abs(Minv - Ainv).max() <= 1e-11 * np.abs(Ainv).max()
    p = tiny("adaptive", tau=1e-6, element="Q1E")
    out = pcg.solve(BDDC(p), p.f[0], rtol=1e-10)
    assert out["iters"] <= 1
    p = tiny("corners", nx=16, ns=4, levels=3, groups=(1, 1), element="Q1E")
    M3 = BDDC(p).dense_preconditioner()
    M2 = BDDC(p, levels=2).dense_preconditioner()
    assert np.abs(M3 - M2).max() <= 1e-11 * np.abs(M2).max()


def test_elasticity_adaptive_setup_meets_target():
    """Theorem "adaptive" on elasticity, three levels: every level's omega <= tau,
    the indicator <= tau^(L-1), and the spectrum within the product of the
    levels' omegas (computed by brute force)."""
    tau = 3.0
    p = tiny("adaptive", nx=16, ns=4, levels=3, groups=(2, 2), tau=tau, seed=3, element="Q1E")
    B = BDDC(p)
    assert all(w <= tau for w in B.omega_levels)
    assert B.indicator <= tau ** (p.levels - 1)
    ev = _dense_MA_eigs(B)
    assert ev[0] >= 1.0 - 1e-10
    om = [_brute_omega(lv) for lv in B.levels]
    assert ev[-1] <= np.prod(om) * (1 + 1e-10)
    Bc = BDDC(p, constraints="corners")
    assert _dense_MA_eigs(Bc)[-1] > ev[-1]
