"""Oracle: multilevel BDDC preconditioner, setup and apply (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see oracle/fem.py).

Setup follows Section 2 (spaces W, U, W-tilde, coarse dofs, E, Q_P, R, R_c),
Section 2.1 (level-l elements are level-(l-1) substructures, level-l dofs are
level-(l-1) coarse dofs, energy-minimal coarse basis functions) and the
adaptive setup algorithm of Section 5 (per level: initial corners, per-edge
eigenproblems, new coarse dofs, then the level's BDDC structures; the last
level is factored directly).

The apply is Algorithm "Multilevel BDDC" of Section 2.1, written out step by
step: interior pre-correction (ML-uIi), residual update (ML-rBi), substructure
correction (ML-wDi), coarse right-hand side (ML-coarse, ML-ri+1), recursion or
direct coarse solve, averaging (ML-uBi-1), interior post-correction (ML-vIi)
and combination (ML-ui).

Local problems are solved as full KKT systems
    [K_i  C_i^T] [w ]   [g]
    [C_i  0    ] [mu] = [0]
with a dense LU factorisation; the coarse basis Psi_i solves the same system
with right-hand side [0; I], and the coarse element matrix is Psi_i^T K_i Psi_i.

Readings where the paper is silent (each also listed in the design doc):
  * stiffness scaling: delta_i(x) = K_i(x,x) / sum_{j in N_x} K_j(x,x) on the
    interface, 1 in the interior; same rule at every level;
  * W-tilde: the values of every global coarse dof agree across the
    substructures that share it (this is C R = R_c Q_P^T of Section 2);
  * edge averages: weight 1/|E| on every dof of the edge;
  * adaptive constraints: per edge, the selected c^s blocks, orthonormalised
    by a QR factorisation (the space W-tilde depends only on their span).
"""

from __future__ import annotations

from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem
from .topology import classify


def assemble_elements(n: int, elems) -> sp.csr_matrix:
    rows, cols, vals = [], [], []
    for dofs, Ke in elems:
        m = len(dofs)
        rows.append(np.repeat(dofs, m))
        cols.append(np.tile(dofs, m))
        vals.append(np.asarray(Ke).reshape(-1))
    if not rows:
        return sp.csr_matrix((n, n))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


class Level:
    """One decomposition level l: level-l elements grouped into substructures."""

    def __init__(self, ell: int, n: int, elems, elem_sub, nsub: int,
                 elem_floating, z: np.ndarray, comp: Optional[np.ndarray] = None):
        self.ell = ell
        self.n = n
        # displacement component of each dof (0 for scalar problems; -1 for a
        # coarse dof that mixes components, as adaptive constraints do)
        self.comp = np.zeros(n, dtype=np.int64) if comp is None else np.asarray(comp, dtype=np.int64)
        self.elems = elems
        self.elem_sub = np.asarray(elem_sub)
        self.nsub = nsub
        self.z = np.asarray(z).reshape(n, -1)   # the kernel's modes (columns) on the level's dofs
        self.A = assemble_elements(n, elems)
        self.topo = classify(n, elems, self.elem_sub, nsub, np.asarray(elem_floating))
        self._local_matrices()
        self._weights()
        int_dofs = np.nonzero(self.topo.interior)[0]
        self.int_dofs = int_dofs
        if len(int_dofs):
            AII = self.A[int_dofs][:, int_dofs].tocsc()
            self.AII_lu = spla.splu(AII)
        else:
            self.AII_lu = None

    # ----- local Neumann matrices K_i (Section 2: a is assembled from them)
    def _local_matrices(self):
        by_sub = [[] for _ in range(self.nsub)]
        for e, s in enumerate(self.elem_sub):
            by_sub[int(s)].append(e)
        self.K = []
        for s in range(self.nsub):
            loc = self.topo.local[s]
            Ks = np.zeros((len(loc), len(loc)))
            for e in by_sub[s]:
                dofs, Ke = self.elems[e]
                p = np.searchsorted(loc, dofs)
                Ks[np.ix_(p, p)] += Ke
            self.K.append(Ks)

    # ----- stiffness-scaling weights (E = sum_i R_i^T D_i, E R = I)
    def _weights(self):
        dsum = np.zeros(self.n)
        for s in range(self.nsub):
            np.add.at(dsum, self.topo.local[s], np.diag(self.K[s]))
        self.delta = []
        for s in range(self.nsub):
            loc = self.topo.local[s]
            d = np.diag(self.K[s]) / dsum[loc]
            d = np.where(self.topo.interior[loc], 1.0, d)
            self.delta.append(d)

    def interface_positions(self, s: int) -> np.ndarray:
        return np.nonzero(~self.topo.interior[self.topo.local[s]])[0]

    def schur(self, s: int) -> np.ndarray:
        """Dense Schur complement of K_s onto its interface dofs."""
        return schur_onto(self.K[s], self.interface_positions(s))

    # ----- coarse dofs: columns of Q_P as (support dofs, weights)
    def build_coarse(self, kind: str, edge_Q: Optional[dict] = None):
        top = self.topo
        func = []
        owners = []
        comp_next = []
        for c in top.corners:
            func.append((np.array([c]), np.array([1.0])))
            owners.append(top.N[c])
            comp_next.append(self.comp[c])
        for key, E in top.edges.items():
            if kind == "corners_edges":
                # the arithmetic average over the edge of each displacement
                # component (Table 1: c+e adds two coarse dofs per edge in 2D
                # elasticity), components in increasing order
                for c in np.unique(self.comp[E]):
                    Ec = E[self.comp[E] == c]
                    func.append((Ec, np.full(len(Ec), 1.0 / len(Ec))))
                    owners.append(key)
                    comp_next.append(c)
            elif kind == "adaptive":
                Q = edge_Q.get(key) if edge_Q else None
                if Q is not None:
                    for m in range(Q.shape[1]):
                        func.append((E, Q[:, m].copy()))
                        owners.append(key)
                        comp_next.append(-1)
        self.func = func
        self.comp_next = np.array(comp_next, dtype=np.int64)
        self.Nc = len(func)
        sub_c = [[] for _ in range(self.nsub)]
        for k, ow in enumerate(owners):
            for s in ow:
                sub_c[s].append(k)
        self.cids = [np.array(v, dtype=np.int64) for v in sub_c]
        self.C, self.kkt, self.Psi, self.Ac = [], [], [], []
        for s in range(self.nsub):
            loc = top.local[s]
            nc = len(self.cids[s])
            C = np.zeros((nc, len(loc)))
            for r, k in enumerate(self.cids[s]):
                dofs, w = func[k]
                C[r, np.searchsorted(loc, dofs)] = w
            n = len(loc)
            M = np.zeros((n + nc, n + nc))
            M[:n, :n] = self.K[s]
            M[:n, n:] = C.T
            M[n:, :n] = C
            lu = sla.lu_factor(M)
            rhs = np.zeros((n + nc, nc))
            rhs[n:, :] = np.eye(nc)
            Psi = sla.lu_solve(lu, rhs)[:n, :]
            self.C.append(C)
            self.kkt.append(lu)
            self.Psi.append(Psi)
            self.Ac.append(Psi.T @ self.K[s] @ Psi)
        self.z_next = np.array([w @ self.z[d] for d, w in func]).reshape(len(func), self.z.shape[1])

    def local_solve(self, s: int, g: np.ndarray) -> np.ndarray:
        """w in W_Delta,s: min 1/2 w^T K_s w - g^T w subject to C_s w = 0 (eq. ML-wDi)."""
        n = len(g)
        nc = self.C[s].shape[0]
        rhs = np.concatenate([g, np.zeros(nc)])
        return sla.lu_solve(self.kkt[s], rhs)[:n]

    def interior_solve(self, r: np.ndarray) -> np.ndarray:
        u = np.zeros(self.n)
        if self.AII_lu is not None:
            u[self.int_dofs] = self.AII_lu.solve(r[self.int_dofs])
        return u


def schur_onto(K: np.ndarray, keep: np.ndarray) -> np.ndarray:
    keep = np.asarray(keep)
    rest = np.setdiff1d(np.arange(K.shape[0]), keep)
    Kkk = K[np.ix_(keep, keep)]
    if len(rest) == 0:
        return Kkk.copy()
    Krr = K[np.ix_(rest, rest)]
    Kkr = K[np.ix_(keep, rest)]
    S = Kkk - Kkr @ np.linalg.solve(Krr, Kkr.T)
    return 0.5 * (S + S.T)


class BDDC:
    """Adaptive-multilevel BDDC built from a synth.Problem-like object."""

    def __init__(self, prob, constraints: Optional[str] = None, tau: Optional[float] = None,
                 levels: Optional[int] = None, all_interface_corners: bool = False):
        self.prob = prob
        self.kind = constraints or prob.constraints
        self.tau = prob.tau if tau is None else tau
        self.L = prob.levels if levels is None else levels
        nx, ny = prob.nx, prob.ny
        self.A = fem.assemble(nx, ny, prob.coeff, prob.element)
        elems, touches = fem.level1_elements(nx, ny, prob.coeff, prob.element)
        n = fem.n_free(nx, ny, prob.element)
        self.levels: List[Level] = []
        self.eigs = []                       # per level: {(s,t): lambdas}
        self.edge_Q = []                     # per level: {(s,t): orthonormal constraint columns}
        self.omega_levels = []               # per level: max_st lambda_{n+1}
        cur = Level(1, n, elems, prob.part, prob.nsub, ~touches, fem.null_modes(nx, ny, prob.element),
                    fem.dof_components(nx, ny, prob.element))
        from . import adaptive
        for ell in range(1, self.L):
            if all_interface_corners and ell == 1:
                top = cur.topo
                top.corners = np.nonzero(~top.interior)[0]
                top.edges = {}
            edge_Q = None
            if self.kind == "adaptive":
                edge_Q, lam, omega = adaptive.select_level(cur, self.tau)
                self.eigs.append(lam)
                self.edge_Q.append(edge_Q)
                self.omega_levels.append(omega)
            cur.build_coarse(self.kind, edge_Q)
            self.levels.append(cur)
            if ell < self.L - 1:
                nxt_elems = [(cur.cids[s], cur.Ac[s]) for s in range(cur.nsub)]
                agg = np.asarray(prob.agglom[ell - 1])
                nsub_next = int(agg.max()) + 1
                cur = Level(ell + 1, cur.Nc, nxt_elems, agg, nsub_next,
                            cur.topo.sub_floating, cur.z_next, cur.comp_next)
        last = self.levels[-1]
        Ac = assemble_elements(last.Nc, [(last.cids[s], last.Ac[s]) for s in range(last.nsub)])
        self.A_coarsest = Ac.toarray()
        self.coarse_chol = sla.cho_factor(self.A_coarsest) if last.Nc else None

    @property
    def indicator(self) -> float:
        return float(np.prod(self.omega_levels)) if self.omega_levels else float("nan")

    def nc_per_level(self):
        return [lv.Nc for lv in self.levels]

    # ----- Algorithm "Multilevel BDDC"
    def _apply_level(self, li: int, r: np.ndarray) -> np.ndarray:
        lv = self.levels[li]
        uI = lv.interior_solve(r)                                    # ML-uIi
        rB = r - lv.A @ uI                                           # ML-rBi
        loc = lv.topo.local
        g = [lv.delta[s] * rB[loc[s]] for s in range(lv.nsub)]     # D_i R_i r_B
        wD = [lv.local_solve(s, g[s]) for s in range(lv.nsub)]     # ML-wDi
        rc = np.zeros(lv.Nc)                                         # ML-coarse / ML-ri+1
        for s in range(lv.nsub):
            np.add.at(rc, lv.cids[s], lv.Psi[s].T @ g[s])
        if li == len(self.levels) - 1:
            uc = sla.cho_solve(self.coarse_chol, rc) if lv.Nc else rc
        else:
            uc = self._apply_level(li + 1, rc)
        uB = np.zeros(lv.n)                                          # ML-uBi-1
        for s in range(lv.nsub):
            w = wD[s] + lv.Psi[s] @ uc[lv.cids[s]]
            np.add.at(uB, loc[s], lv.delta[s] * w)
        vI = lv.interior_solve(lv.A @ uB)                            # ML-vIi
        return uI + uB - vI                                          # ML-ui

    def apply(self, r: np.ndarray) -> np.ndarray:
        return self._apply_level(0, np.asarray(r, dtype=np.float64))

    def condensed_x0(self, b: np.ndarray) -> np.ndarray:
        """Interface-reduced start: interior values solve A_II x_I = b_I, interface 0."""
        return self.levels[0].interior_solve(b)

    def dense_preconditioner(self) -> np.ndarray:
        n = self.levels[0].n
        return np.column_stack([self.apply(np.eye(n)[:, j]) for j in range(n)])
