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

Elasticity ("Q1E", the problem of the paper's numerical section): plane
strain with Lame parameters lambda = 1, mu = 2 scaled per element by k_e,
a(u, v) = sum_e k_e int_e eps(u) : C eps(v), eps(u) = sym grad u, Q1 for both
displacement components, two dofs per node (x then y), the whole boundary
clamped.  The element matrix is the 2x2 Gauss quadrature of B^T D B (exact
for bilinear fields on rectangles), with D the plane-strain elasticity matrix
in engineering shear strain.
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


LAME_LAMBDA = 1.0
LAME_MU = 2.0


def elasticity_d(lam: float = LAME_LAMBDA, mu: float = LAME_MU) -> np.ndarray:
    """Plane strain: sigma = D (eps_xx, eps_yy, gamma_xy), gamma_xy = 2 eps_xy."""
    return np.array([[lam + 2 * mu, lam, 0.0],
                     [lam, lam + 2 * mu, 0.0],
                     [0.0, 0.0, mu]])


def q1_elastic_element_matrix(hx: float, hy: float, lam: float = LAME_LAMBDA,
                              mu: float = LAME_MU) -> np.ndarray:
    """int_e eps(phi_a) : C eps(phi_b) over an hx x hy rectangle (k = 1), 2x2
    Gauss; dof 2 a + c is component c (0: x, 1: y) of local node a."""
    D = elasticity_d(lam, mu)
    g = 0.5 / np.sqrt(3.0)
    pts = [0.5 - g, 0.5 + g]
    K = np.zeros((8, 8))
    for xi in pts:
        for eta in pts:
            dxi, deta = _q1_grad(xi, eta)
            gx = dxi / hx
            gy = deta / hy
            B = np.zeros((3, 8))
            B[0, 0::2] = gx          # eps_xx = du_x/dx
            B[1, 1::2] = gy          # eps_yy = du_y/dy
            B[2, 0::2] = gy          # gamma_xy = du_x/dy + du_y/dx
            B[2, 1::2] = gx
            K += 0.25 * hx * hy * (B.T @ D @ B)
    return K


def dofs_per_node(element: str) -> int:
    return 2 if element == "Q1E" else 1


def element_matrix(element: str, nx: int, ny: int) -> np.ndarray:
    hx, hy = 1.0 / nx, 1.0 / ny
    if element == "Q1":
        return q1_element_matrix(hx, hy)
    if element == "P1":
        return p1_element_matrix(hx, hy)
    if element == "Q1E":
        return q1_elastic_element_matrix(hx, hy)
    raise ValueError(element)


def free_index(nx: int, ny: int) -> np.ndarray:
    """(ny+1) x (nx+1) grid of node -> free dof index, -1 on the boundary."""
    idx = -np.ones((ny + 1, nx + 1), dtype=np.int64)
    idx[1:ny, 1:nx] = np.arange((nx - 1) * (ny - 1)).reshape(ny - 1, nx - 1)
    return idx


def element_dofs(nx: int, ny: int, element: str = "Q1") -> np.ndarray:
    """(nx*ny, m) free dof of each element dof in local order, -1 for Dirichlet
    nodes: m = 4 nodes, or for elasticity m = 8 (free node f has dofs 2 f and
    2 f + 1)."""
    idx = free_index(nx, ny)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    i = i.reshape(-1)
    j = j.reshape(-1)
    nodes = np.stack([idx[j, i], idx[j, i + 1], idx[j + 1, i + 1], idx[j + 1, i]], axis=1)
    if dofs_per_node(element) == 1:
        return nodes
    out = np.empty((nodes.shape[0], 8), dtype=np.int64)
    out[:, 0::2] = np.where(nodes >= 0, 2 * nodes, -1)
    out[:, 1::2] = np.where(nodes >= 0, 2 * nodes + 1, -1)
    return out


def n_free(nx: int, ny: int, element: str = "Q1") -> int:
    return dofs_per_node(element) * (nx - 1) * (ny - 1)


def dof_components(nx: int, ny: int, element: str = "Q1") -> np.ndarray:
    """Displacement component of each free dof: 0 for scalar problems; for
    elasticity 0 (x) on dofs 2 f and 1 (y) on dofs 2 f + 1."""
    return np.arange(n_free(nx, ny, element), dtype=np.int64) % dofs_per_node(element)


def null_modes(nx: int, ny: int, element: str = "Q1") -> np.ndarray:
    """(n_free, m) the kernel of the operator without Dirichlet data, on the
    free dofs: the constants (scalar problems, m = 1) or the rigid-body modes
    of plane elasticity (m = 3: the two translations and the infinitesimal
    rotation u = (-y, x), at the node coordinates)."""
    nf = (nx - 1) * (ny - 1)
    if dofs_per_node(element) == 1:
        return np.ones((nf, 1))
    f = np.arange(nf)
    x = (f % (nx - 1) + 1) / nx
    y = (f // (nx - 1) + 1) / ny
    Z = np.zeros((2 * nf, 3))
    Z[0::2, 0] = 1.0
    Z[1::2, 1] = 1.0
    Z[0::2, 2] = -y
    Z[1::2, 2] = x
    return Z


def assemble(nx: int, ny: int, coeff: np.ndarray, element: str = "Q1") -> sp.csr_matrix:
    """Global stiffness A over the free dofs: A = sum_e k_e * R_e^T K_hat R_e."""
    Kh = element_matrix(element, nx, ny)
    dofs = element_dofs(nx, ny, element)
    m_e = dofs.shape[1]
    rows, cols, vals = [], [], []
    for a in range(m_e):
        for b in range(m_e):
            m = (dofs[:, a] >= 0) & (dofs[:, b] >= 0)
            rows.append(dofs[m, a])
            cols.append(dofs[m, b])
            vals.append(coeff[m] * Kh[a, b])
    n = n_free(nx, ny, element)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return A.tocsr()


def level1_elements(nx: int, ny: int, coeff: np.ndarray, element: str = "Q1"):
    """Level-1 'elements' in the generic form used by the multilevel oracle:
    a list of (dof array, element matrix) with Dirichlet nodes removed, and a
    flag telling whether the element touches the Dirichlet boundary."""
    Kh = element_matrix(element, nx, ny)
    dofs = element_dofs(nx, ny, element)
    elems = []
    touches = np.zeros(nx * ny, dtype=bool)
    for e in range(nx * ny):
        keep = dofs[e] >= 0
        touches[e] = not keep.all()
        elems.append((dofs[e][keep].copy(), coeff[e] * Kh[np.ix_(keep, keep)]))
    return elems, touches
