"""Pins of the assembled operator, the stencil application and the Thomas solver."""

import numpy as np
import pytest

from oracle.operator import apply_laplacian, assemble_matrix, backward_error
from oracle.thomas import thomas, thomas_cyclic


def test_assembled_1d_by_hand():
    # 3 cells, unit spacing.  Dirichlet ends: ghost -u0 -> diagonal -3; Neumann: -1; periodic wraps.
    D = assemble_matrix((1, 1, 3), "DDPPPP", (1.0, 1.0, 1.0))
    np.testing.assert_array_equal(D, [[-3, 1, 0], [1, -2, 1], [0, 1, -3]])
    N = assemble_matrix((1, 1, 3), "NNPPPP", (1.0, 1.0, 1.0))
    np.testing.assert_array_equal(N, [[-1, 1, 0], [1, -2, 1], [0, 1, -1]])
    P = assemble_matrix((1, 1, 3), "PPPPPP", (1.0, 1.0, 1.0))
    np.testing.assert_array_equal(P, [[-2, 1, 1], [1, -2, 1], [1, 1, -2]])
    # mixed z faces (Dirichlet below, Neumann above), spacing 0.5 in z
    Z = assemble_matrix((3, 1, 1), "PPPPDN", (1.0, 1.0, 0.5))
    np.testing.assert_array_equal(Z, 4.0 * np.array([[-3, 1, 0], [1, -2, 1], [0, 1, -1]]))


@pytest.mark.parametrize("bc", ["PPPPDD", "DDNNNN", "PPPPNN", "NNDDPP", "DDDDDN"])
def test_assembled_matches_stencil_and_kronecker(bc):
    shape = (3, 4, 5)
    h = (0.7, 1.3, 0.9)
    A = assemble_matrix(shape, bc, h)
    u = np.random.default_rng(0).standard_normal(shape)
    np.testing.assert_allclose(A @ u.reshape(-1), apply_laplacian(u, bc, h).reshape(-1), atol=1e-12)
    # Kronecker sum of the 1-D operators (x fastest)
    Ax = assemble_matrix((1, 1, 5), bc[0:2] + "PPPP", (h[0], 1, 1))
    Ay = assemble_matrix((1, 1, 4), bc[2:4] + "PPPP", (h[1], 1, 1))
    Az = assemble_matrix((1, 1, 3), bc[4:6] + "PPPP", (h[2], 1, 1))
    K = (np.kron(Az, np.eye(20)) + np.kron(np.eye(3), np.kron(Ay, np.eye(5)))
         + np.kron(np.eye(12), Ax))
    np.testing.assert_allclose(A, K, atol=1e-12)
    np.testing.assert_allclose(A, A.T, atol=0)          # symmetric for homogeneous faces


@pytest.mark.parametrize("bc,singular", [("PPPPNN", True), ("NNNNNN", True), ("PPNNPP", True),
                                         ("PPPPDD", False), ("DDNNNN", False), ("NNNNDN", False)])
def test_null_space(bc, singular):
    A = assemble_matrix((3, 2, 4), bc, (1.0, 0.5, 2.0))
    ones = np.ones(A.shape[0])
    assert (np.max(np.abs(A @ ones)) < 1e-12) == singular
    assert (np.linalg.matrix_rank(A) == A.shape[0] - 1) == singular


def test_thomas_against_dense():
    rng = np.random.default_rng(3)
    for n in [1, 2, 3, 7, 16, 65]:
        a = rng.uniform(0.5, 1.5, (4, n))
        c = rng.uniform(0.5, 1.5, (4, n))
        b = -(np.abs(a) + np.abs(c) + rng.uniform(0.1, 1.0, (4, n)))
        r = rng.standard_normal((4, n)) + 1j * rng.standard_normal((4, n))
        x = thomas(a, b, c, r)
        for s in range(4):
            M = np.diag(b[s]) + np.diag(a[s, 1:], -1) + np.diag(c[s, :-1], 1)
            np.testing.assert_allclose(x[s], np.linalg.solve(M, r[s]), rtol=0, atol=1e-12)


def test_thomas_cyclic_against_dense():
    rng = np.random.default_rng(4)
    for n in [3, 4, 9, 32]:
        a = rng.uniform(0.5, 1.5, n)
        c = rng.uniform(0.5, 1.5, n)
        b = -(a + c + rng.uniform(0.1, 1.0, n))
        r = rng.standard_normal(n)
        M = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
        M[0, n - 1] = a[0]
        M[n - 1, 0] = c[n - 1]
        np.testing.assert_allclose(thomas_cyclic(a, b, c, r), np.linalg.solve(M, r), atol=1e-12)


def test_backward_error_small_for_exact_and_large_for_wrong():
    bc, h = "DDDDDD", (0.5, 0.5, 0.5)
    A = assemble_matrix((3, 3, 3), bc, h)
    f = np.random.default_rng(5).standard_normal((3, 3, 3))
    u = np.linalg.solve(A, f.reshape(-1)).reshape(f.shape)
    assert backward_error(f, u, bc, h) < 1e-15
    assert backward_error(f, 1.01 * u, bc, h) > 1e-4
