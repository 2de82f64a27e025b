"""Pins of the oracle's discretisation against closed forms (no GPU)."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem


def test_q1_square_element_closed_form():
    # bilinear element on a square: diagonal 2/3, side neighbours -1/6, opposite -1/3
    K = fem.q1_element_matrix(0.25, 0.25)
    ref = np.array([[4, -1, -2, -1], [-1, 4, -1, -2], [-2, -1, 4, -1], [-1, -2, -1, 4]]) / 6.0
    assert np.allclose(K, ref, atol=1e-15)


@pytest.mark.parametrize("hx,hy", [(0.5, 0.25), (0.1, 0.3)])
def test_q1_rectangle_energy_of_linear_functions(hx, hy):
    K = fem.q1_element_matrix(hx, hy)
    x = np.array([0.0, hx, hx, 0.0])     # u = x on the element
    y = np.array([0.0, 0.0, hy, hy])     # u = y
    one = np.ones(4)
    # int |grad x|^2 = area, int grad x . grad y = 0, constants have no energy
    assert np.isclose(x @ K @ x, hx * hy, rtol=1e-14)
    assert np.isclose(y @ K @ y, hx * hy, rtol=1e-14)
    assert abs(x @ K @ y) < 1e-15
    assert np.allclose(K @ one, 0.0, atol=1e-14)
    # u = x*y is bilinear, hence in the element space: int |grad(xy)|^2 = hx hy (hx^2 + hy^2) / 3
    xy = np.array([0.0, 0.0, hx * hy, 0.0])
    assert np.isclose(xy @ K @ xy, hx * hy * (hx**2 + hy**2) / 3.0, rtol=1e-13)


def test_p1_square_is_five_point_stencil():
    K = fem.p1_element_matrix(1.0, 1.0)
    ref = 0.5 * np.array([[2, -1, 0, -1], [-1, 2, -1, 0], [0, -1, 2, -1], [-1, 0, -1, 2]])
    assert np.allclose(K, ref, atol=1e-15)
    A = fem.assemble(6, 6, np.ones(36), "P1").toarray()
    c = 2 * 5 + 2                          # free node (3,3)
    row = A[c]
    assert np.isclose(row[c], 4.0)
    assert np.isclose(row.sum() - row[c], -4.0)


def test_q1_assembled_nine_point_stencil():
    nx = 6
    A = fem.assemble(nx, nx, np.ones(nx * nx), "Q1").toarray()
    c = 2 * (nx - 1) + 2
    row = A[c]
    nz = np.sort(row[np.abs(row) > 1e-14])
    assert np.isclose(row[c], 8.0 / 3.0)
    assert len(nz) == 9
    assert np.allclose(nz[:8], -1.0 / 3.0)
    assert np.allclose(A, A.T)


def test_manufactured_direct_solve():
    rng = np.random.default_rng(3)
    nx = 20
    k = 10 ** rng.uniform(0, 4, nx * nx)
    A = fem.assemble(nx, nx, k, "Q1").tocsc()
    um = rng.standard_normal(A.shape[0])
    b = A @ um
    u = spla.spsolve(A, b)
    assert np.linalg.norm(u - um) / np.linalg.norm(um) < 1e-11


def test_element_dofs_layout():
    nx = 4
    d = fem.element_dofs(nx, nx)
    # element (1,1) has nodes (1,1),(2,1),(2,2),(1,2) -> free ids 0,1,4,3
    assert list(d[1 * nx + 1]) == [0, 1, 4, 3]
    # the corner element touches three Dirichlet nodes
    assert list(d[0]) == [-1, -1, 0, -1]


# ---------------------------------------------------------------- elasticity (the paper's experiments)
def _rigid_modes(hx, hy):
    x = np.array([0.0, hx, hx, 0.0])
    y = np.array([0.0, 0.0, hy, hy])
    tx = np.zeros(8)
    tx[0::2] = 1.0
    ty = np.zeros(8)
    ty[1::2] = 1.0
    rot = np.zeros(8)                    # u = (-y, x): an infinitesimal rotation
    rot[0::2] = -y
    rot[1::2] = x
    return x, y, [tx, ty, rot]


@pytest.mark.parametrize("hx,hy", [(0.25, 0.25), (0.5, 0.2)])
def test_elastic_element_null_space_is_the_rigid_modes(hx, hy):
    K = fem.q1_elastic_element_matrix(hx, hy)
    assert np.allclose(K, K.T, atol=1e-14)
    _, _, Z = _rigid_modes(hx, hy)
    for z in Z:
        assert np.abs(K @ z).max() <= 1e-13 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev > 1e-10 * ev[-1]) == 5      # 8 dofs - 3 rigid modes
    assert ev[0] >= -1e-13 * ev[-1]


@pytest.mark.parametrize("hx,hy", [(0.25, 0.25), (0.5, 0.2)])
def test_elastic_element_energy_of_linear_and_bilinear_fields(hx, hy):
    """Bilinear elements hold every linear field exactly, so u^T K u is the
    exact strain energy int eps : C eps: for a constant strain (e_xx, e_yy,
    gamma) it is (e^T D e) hx hy with plane-strain D (lambda = 1, mu = 2);
    u = (x y, 0) is bilinear too: eps_xx = y, gamma = x."""
    lam, mu = fem.LAME_LAMBDA, fem.LAME_MU
    K = fem.q1_elastic_element_matrix(hx, hy)
    x, y, _ = _rigid_modes(hx, hy)
    D = np.array([[lam + 2 * mu, lam, 0.0], [lam, lam + 2 * mu, 0.0], [0.0, 0.0, mu]])
    rng = np.random.default_rng(3)
    for _ in range(4):
        a, b, c, d = rng.standard_normal(4)     # u = (a x + b y, c x + d y)
        u = np.zeros(8)
        u[0::2] = a * x + b * y
        u[1::2] = c * x + d * y
        e = np.array([a, d, b + c])
        assert np.isclose(u @ K @ u, e @ D @ e * hx * hy, rtol=1e-13)
    u = np.zeros(8)
    u[0::2] = x * y
    ref = (lam + 2 * mu) * hx * hy**3 / 3.0 + mu * hy * hx**3 / 3.0
    assert np.isclose(u @ K @ u, ref, rtol=1e-13)


def test_elastic_patch_test_reproduces_a_linear_field():
    """Clamp the boundary nodes of a 7 x 5 grid of one material to a linear
    displacement field and solve for the interior (no body force): the FE
    solution is that field at every interior node.  Also checks the assembly
    of the free dofs (two per node, 2 f + c), with element-wise coefficients,
    against the all-node matrix built here."""
    nx, ny = 7, 5
    hx, hy = 1.0 / nx, 1.0 / ny
    Ke = fem.q1_elastic_element_matrix(hx, hy)
    nn = (nx + 1) * (ny + 1)

    def full_matrix(kcoef):
        full = np.zeros((2 * nn, 2 * nn))
        for j in range(ny):
            for i in range(nx):
                nodes = [j * (nx + 1) + i, j * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i + 1,
                         (j + 1) * (nx + 1) + i]
                dof = np.ravel([[2 * a, 2 * a + 1] for a in nodes])
                full[np.ix_(dof, dof)] += kcoef[j * nx + i] * Ke
        return full
    X, Y = np.meshgrid(np.arange(nx + 1) * hx, np.arange(ny + 1) * hy)
    X, Y = X.ravel(), Y.ravel()
    ulin = np.zeros(2 * nn)
    ulin[0::2] = 0.3 + 1.5 * X - 0.7 * Y
    ulin[1::2] = -0.2 + 0.4 * X + 2.0 * Y
    interior = np.zeros(nn, dtype=bool)
    for j in range(1, ny):
        for i in range(1, nx):
            interior[j * (nx + 1) + i] = True
    I = np.ravel([[2 * a, 2 * a + 1] for a in np.nonzero(interior)[0]])
    B = np.setdiff1d(np.arange(2 * nn), I)
    # the oracle's free-dof matrix is the interior block, in the same order
    kvar = 10.0 ** np.random.default_rng(5).uniform(0, 2, nx * ny)
    A = fem.assemble(nx, ny, kvar, "Q1E").toarray()
    assert A.shape == (len(I), len(I))
    assert np.abs(A - full_matrix(kvar)[np.ix_(I, I)]).max() <= 1e-12 * np.abs(A).max()
    kone = np.full(nx * ny, 3.0)
    full = full_matrix(kone)
    A = fem.assemble(nx, ny, kone, "Q1E").toarray()
    uI = np.linalg.solve(A, -full[np.ix_(I, B)] @ ulin[B])
    assert np.abs(uI - ulin[I]).max() <= 1e-12
