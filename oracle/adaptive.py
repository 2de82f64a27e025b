"""Oracle: per-edge generalized eigenproblems of the adaptive setup.

TEST INFRASTRUCTURE ONLY (see oracle/fem.py).

For adjacent level-l substructures s, t (they share an edge) the pair space
lives on the interface dofs of s and of t, kept as separate copies
w = (w_s, w_t), with S = blkdiag(S_s, S_t) the Schur complements of the local
matrices onto their interfaces (Section 3).  Theorem "local-est":
    X = Pi (I-E)^T S (I-E) Pi,
    Y = Pib (Pi S Pi + a (I-Pi)) Pib + a (I-Pib),
with Pi the orthogonal projection onto the null space of the initial
constraints C (I-E) (here: equal values of the shared corners), and I-Pib the
orthogonal projection onto null(Pi S Pi + a (I-Pi)), built from a matrix Z whose
range holds the null space of S (the constant on each floating substructure at
level 1, the coarse-dof values of the constant at higher levels).

(I-E) is the pair averaging complement: on a shared dof x the s-copy row is
delta_t(x) (e_s(x) - e_t(x)) and the t-copy row delta_s(x) (e_t(x) - e_s(x)),
with the pair weights delta_s = d_s / (d_s + d_t) built locally so that
E^{st} R^{st} = I (Section 5); other rows are zero.

Selection (Section 5, adaptive setup; Theorem "adaptive"): eigenvalues are
sorted in decreasing order and every eigenvector with lambda > tau is used.
The constraint row is c_k = w_k^T X (eq. generate-constraints); c^s = -c^t,
so the s block restricted to the edge dofs is kept and becomes a new coarse
dof q_k = R^{sT} c^{sT}.  Reading: the strict rule lambda > tau, which is the
one consistent with the counts of Table 6 against Table 3.
The edge indicator is the largest unselected eigenvalue; the level value is
the maximum over edges and the indicator omega-tilde is the product over
levels (eq. cond-est).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .bddc import schur_onto

QR_DROP = 1e-10


def _pair_setup(level, s, t):
    top = level.topo
    gs = level.interface_positions(s)
    gt = level.interface_positions(t)
    ds_glob = top.local[s][gs]
    dt_glob = top.local[t][gt]
    F = np.intersect1d(ds_glob, dt_glob)
    ps = {int(d): i for i, d in enumerate(ds_glob)}
    pt = {int(d): len(gs) + i for i, d in enumerate(dt_glob)}
    diag_s = np.diag(level.K[s])[gs]
    diag_t = np.diag(level.K[t])[gt]
    return gs, gt, ds_glob, dt_glob, F, ps, pt, diag_s, diag_t


def _projections(n, G, Z):
    I = np.eye(n)
    if G.shape[0]:
        Pi = I - G.T @ np.linalg.pinv(G @ G.T) @ G
    else:
        Pi = I.copy()
    if Z.shape[1]:
        N0 = sla.null_space(G @ Z) if G.shape[0] else np.eye(Z.shape[1])
        if N0.shape[1]:
            Q = sla.orth(Z @ N0)
            Pib = I - Q @ Q.T
        else:
            Pib = I.copy()
    else:
        Pib = I.copy()
    return Pi, Pib


def pair_eig_full(level, s, t, extra_rows=None):
    """Full-form pair eigenproblem of Theorem "local-est".

    extra_rows: optional list of constraint vectors c (on the edge dofs) added
    as rows [c on s-edge, -c on t-edge] to C(I-E).
    Returns (lam_desc, V, X, info) with V the Y-orthonormal eigenvectors.
    """
    top = level.topo
    gs, gt, ds_glob, dt_glob, F, ps, pt, diag_s, diag_t = _pair_setup(level, s, t)
    n = len(gs) + len(gt)
    S = sla.block_diag(level.schur(s), level.schur(t))
    IE = np.zeros((n, n))
    for d in F:
        i, j = ps[int(d)], pt[int(d)]
        a, b = diag_s[i], diag_t[j - len(gs)]
        dls, dlt = a / (a + b), b / (a + b)
        IE[i, i] += dlt
        IE[i, j] -= dlt
        IE[j, j] += dls
        IE[j, i] -= dls
    cset = set(int(c) for c in top.corners)
    rows = []
    for d in F:
        if int(d) in cset:
            r = np.zeros(n)
            r[ps[int(d)]] = 1.0
            r[pt[int(d)]] = -1.0
            rows.append(r)
    E = top.edges[(s, t)]
    if extra_rows:
        for c in extra_rows:
            r = np.zeros(n)
            r[[ps[int(d)] for d in E]] = c
            r[[pt[int(d)] for d in E]] = -c
            rows.append(r)
    G = np.array(rows).reshape(len(rows), n)
    # the kernels of the floating substructures' operators (one column per
    # mode: the constants, or the rigid-body modes of elasticity)
    zcols = []
    if top.sub_floating[s]:
        for m in range(level.z.shape[1]):
            zc = np.zeros(n)
            zc[:len(gs)] = level.z[ds_glob, m]
            zcols.append(zc)
    if top.sub_floating[t]:
        for m in range(level.z.shape[1]):
            zc = np.zeros(n)
            zc[len(gs):] = level.z[dt_glob, m]
            zcols.append(zc)
    Z = np.array(zcols).T.reshape(n, len(zcols))
    Pi, Pib = _projections(n, G, Z)
    X = Pi @ IE.T @ S @ IE @ Pi
    X = 0.5 * (X + X.T)
    a = float(np.max(np.diag(S)))
    Y = Pib @ (Pi @ S @ Pi + a * (np.eye(n) - Pi)) @ Pib + a * (np.eye(n) - Pib)
    Y = 0.5 * (Y + Y.T)
    lam, V = sla.eigh(X, Y)
    lam = lam[::-1]
    V = V[:, ::-1]
    info = dict(ps=ps, pt=pt, E=E, F=F, n=n)
    return lam, V, X, info


def pair_eig_reduced(level, s, t):
    """Same pencil with the non-shared interface dofs eliminated: the numerator
    keeps the F x F block of S, the denominator becomes the Schur complement of
    each local matrix onto the shared dofs F.  Returns the eigenvalues (desc)."""
    top = level.topo
    gs, gt, ds_glob, dt_glob, F, ps, pt, diag_s, diag_t = _pair_setup(level, s, t)
    nf = len(F)
    n = 2 * nf
    Ss = level.schur(s)
    St = level.schur(t)
    fs = np.array([ps[int(d)] for d in F])
    ft = np.array([pt[int(d)] - len(gs) for d in F])
    Snum = sla.block_diag(Ss[np.ix_(fs, fs)], St[np.ix_(ft, ft)])
    locs = np.searchsorted(top.local[s], F)
    loct = np.searchsorted(top.local[t], F)
    Sden = sla.block_diag(schur_onto(level.K[s], locs), schur_onto(level.K[t], loct))
    IE = np.zeros((n, n))
    for k in range(nf):
        a, b = diag_s[fs[k]], diag_t[ft[k]]
        dls, dlt = a / (a + b), b / (a + b)
        IE[k, k] += dlt
        IE[k, nf + k] -= dlt
        IE[nf + k, nf + k] += dls
        IE[nf + k, k] -= dls
    cset = set(int(c) for c in top.corners)
    rows = []
    for k, d in enumerate(F):
        if int(d) in cset:
            r = np.zeros(n)
            r[k] = 1.0
            r[nf + k] = -1.0
            rows.append(r)
    G = np.array(rows).reshape(len(rows), n)
    zcols = []
    if top.sub_floating[s]:
        for m in range(level.z.shape[1]):
            zc = np.zeros(n)
            zc[:nf] = level.z[F, m]
            zcols.append(zc)
    if top.sub_floating[t]:
        for m in range(level.z.shape[1]):
            zc = np.zeros(n)
            zc[nf:] = level.z[F, m]
            zcols.append(zc)
    Z = np.array(zcols).T.reshape(n, len(zcols))
    Pi, Pib = _projections(n, G, Z)
    X = Pi @ IE.T @ Snum @ IE @ Pi
    X = 0.5 * (X + X.T)
    a = float(np.max(np.diag(Sden)))
    Y = Pib @ (Pi @ Sden @ Pi + a * (np.eye(n) - Pi)) @ Pib + a * (np.eye(n) - Pib)
    Y = 0.5 * (Y + Y.T)
    lam = sla.eigh(X, Y, eigvals_only=True)
    return lam[::-1]


def constraints_from(lam, V, X, info, tau):
    """Selected constraint columns (edge dofs x n_sel) for lambda > tau."""
    E = info["E"]
    ps = info["ps"]
    sel = np.nonzero(lam[:len(E)] > tau)[0]
    cols = []
    for k in sel:
        c = X @ V[:, k]
        cols.append(c[[ps[int(d)] for d in E]])
    return np.array(cols).T.reshape(len(E), len(sel))


def orthonormalise(C):
    if C.shape[1] == 0:
        return C
    Q, R = np.linalg.qr(C)
    dr = np.abs(np.diag(R))
    keep = dr > QR_DROP * dr.max()
    return Q[:, keep]


def select_level(level, tau):
    """Adaptive selection on one level.

    Returns (edge_Q, lam, omega): edge_Q[(s,t)] = orthonormal constraint
    columns on the edge dofs; lam[(s,t)] = the |E| largest eigenvalues; omega
    = max over edges of the largest unselected eigenvalue (0 if none left).
    """
    edge_Q, lams = {}, {}
    omega = 0.0
    for (s, t), E in level.topo.edges.items():
        lam, V, X, info = pair_eig_full(level, s, t)
        lam_e = lam[:len(E)].copy()
        lams[(s, t)] = lam_e
        C = constraints_from(lam, V, X, info, tau)
        edge_Q[(s, t)] = orthonormalise(C)
        nsel = C.shape[1]
        nxt = lam_e[nsel] if nsel < len(lam_e) else 0.0
        omega = max(omega, float(nxt))
    return edge_Q, lams, omega


def indicator_from_tables(per_level_lams, tau):
    """omega-tilde from per-level lists of pair eigenvalues (eq. cond-est with
    the selection rule): product over levels of the max over pairs of the
    largest eigenvalue that is not selected (lambda <= tau)."""
    out = 1.0
    for pairs in per_level_lams:
        best = 0.0
        for lam in pairs:
            rest = [x for x in sorted(lam, reverse=True) if not x > tau]
            if rest:
                best = max(best, rest[0])
        out *= best
    return out


def count_selected(lam, tau):
    return int(sum(1 for x in lam if x > tau))
