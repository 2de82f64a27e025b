"""Oracle: finite element discretisation of the model problem (FP64, CPU).

TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow reference that the
tests, the smoke check and the benchmark's CPU baseline call; the product
path never imports it.

Model problem (Section 2, eq. (problem)): find u in U with a(u, v) = <f, v>
for all v in U, U the continuous Lagrange P1 or Q1 functions that vanish on
the boundary of the unit square, a(u, v) = sum_e k_e * int_e grad u . grad v.

Element matrices are computed from their definition: Q1 by 2x2 Gauss
quadrature of the bilinear shape-function gradients (exact for this
integrand), P1 from the constant gradients of the two triangles of the
element square split along its SW-NE diagonal.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# local node order of an element: (i,j), (i+1,j), (i+1,j+1), (i,j+1)  (counter-clockwise)
_REF_NODES = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])


def _q1_grad(xi, eta):
    """Gradients on the reference square of the four bilinear shape functions."""
    dxi = np.array([-(1 - eta), (1 - eta), eta, -eta])
    deta = np.array([-(1 - xi), -xi, xi, (1 - xi)])
    return dxi, deta


def q1_element_matrix(hx: float, hy: float) -> np.ndarray:
    """int_e grad phi_a . grad phi_b over an hx x hy rectangle (k = 1), 2x2 Gauss."""
    g = 0.5 / np.sqrt(3.0)
    pts = [0.5 - g, 0.5 + g]
    K = np.zeros((4, 4))
    for xi in pts:
        for eta in pts:
            dxi, deta = _q1_grad(xi, eta)
            gx = dxi / hx
            gy = deta / hy
            K += 0.25 * hx * hy * (np.outer(gx, gx) + np.outer(gy, gy))
    return K


def _tri_matrix(xy):
    """P1 stiffness of one triangle with vertices xy (3x2), k = 1."""
    T = np.array([[1.0, xy[0, 0], xy[0, 1]],
                  [1.0, xy[1, 0], xy[1, 1]],
                  [1.0, xy[2, 0], xy[2, 1]]])
    area = 0.5 * abs(np.linalg.det(T))
    coef = np.linalg.inv(T)          # columns: coefficients (c, a, b) of each basis function
    grads = coef[1:3, :].T           # 3 x 2
    return area * grads @ grads.T


def p1_element_matrix(hx: float, hy: float) -> np.ndarray:
    """Sum of the two P1 triangles (SW-NE diagonal) embedded in the 4 square nodes."""
    xy = _REF_NODES * np.array([hx, hy])
    K = np.zeros((4, 4))
    for tri in ([0, 1, 2], [0, 2, 3]):
        Kt = _tri_matrix(xy[tri])
        for a in range(3):
            for b in range(3):
                K[tri[a], tri[b]] += Kt[a, b]
    return K


def element_matrix(element: str, nx: int, ny: int) -> np.ndarray:
    hx, hy = 1.0 / nx, 1.0 / ny
    if element == "Q1":
        return q1_element_matrix(hx, hy)
    if element == "P1":
        return p1_element_matrix(hx, hy)
    raise ValueError(element)


def free_index(nx: int, ny: int) -> np.ndarray:
    """(ny+1) x (nx+1) grid of node -> free dof index, -1 on the boundary."""
    idx = -np.ones((ny + 1, nx + 1), dtype=np.int64)
    idx[1:ny, 1:nx] = np.arange((nx - 1) * (ny - 1)).reshape(ny - 1, nx - 1)
    return idx


def element_dofs(nx: int, ny: int) -> np.ndarray:
    """(nx*ny, 4) free dof of each element node in local order, -1 for Dirichlet nodes."""
    idx = free_index(nx, ny)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    i = i.reshape(-1)
    j = j.reshape(-1)
    return np.stack([idx[j, i], idx[j, i + 1], idx[j + 1, i + 1], idx[j + 1, i]], axis=1)


def assemble(nx: int, ny: int, coeff: np.ndarray, element: str = "Q1") -> sp.csr_matrix:
    """Global stiffness A over the free nodes: A = sum_e k_e * R_e^T K_hat R_e."""
    Kh = element_matrix(element, nx, ny)
    dofs = element_dofs(nx, ny)
    rows, cols, vals = [], [], []
    for a in range(4):
        for b in range(4):
            m = (dofs[:, a] >= 0) & (dofs[:, b] >= 0)
            rows.append(dofs[m, a])
            cols.append(dofs[m, b])
            vals.append(coeff[m] * Kh[a, b])
    n = (nx - 1) * (ny - 1)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return A.tocsr()


def level1_elements(nx: int, ny: int, coeff: np.ndarray, element: str = "Q1"):
    """Level-1 'elements' in the generic form used by the multilevel oracle:
    a list of (dof array, element matrix) with Dirichlet nodes removed, and a
    flag telling whether the element touches the Dirichlet boundary."""
    Kh = element_matrix(element, nx, ny)
    dofs = element_dofs(nx, ny)
    elems = []
    touches = np.zeros(nx * ny, dtype=bool)
    for e in range(nx * ny):
        keep = dofs[e] >= 0
        touches[e] = not keep.all()
        elems.append((dofs[e][keep].copy(), coeff[e] * Kh[np.ix_(keep, keep)]))
    return elems, touches
