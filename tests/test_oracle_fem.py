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
