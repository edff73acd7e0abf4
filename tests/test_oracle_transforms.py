"""Pins of the oracle's transforms and eigenvalues against independent definitions.

Library routines (numpy.fft, scipy.fft) and hand-worked small cases fix the
direct-sum matrices; the eigen-invariant A_1d phi_k = lam_k phi_k ties Table eig,
the transform bases and the ghost rules together.
"""

import numpy as np
import pytest
import scipy.fft as sfft

from oracle import transforms
from oracle.eigen import eigenvalues
from oracle.operator import assemble_matrix

SIZES = [1, 2, 3, 4, 5, 6, 8, 9, 12, 16, 24, 31, 32, 48, 64]


@pytest.mark.parametrize("N", SIZES)
def test_dft_matches_numpy(N):
    x = np.random.default_rng(N).standard_normal(N) + 1j * np.random.default_rng(N + 1).standard_normal(N)
    np.testing.assert_allclose(transforms.dft(N) @ x, np.fft.fft(x), rtol=0, atol=1e-12 * max(1, N))
    np.testing.assert_allclose(transforms.idft(N) @ x, np.fft.ifft(x), rtol=0, atol=1e-13 * max(1, N))


@pytest.mark.parametrize("N", SIZES)
def test_real_transforms_match_scipy(N):
    # scipy's unnormalised types 2 and 3 are twice the paper's Eqs. for DCT10/DCT01/DST10/DST01.
    x = np.random.default_rng(100 + N).standard_normal(N)
    tol = dict(rtol=0, atol=1e-12 * max(1, N))
    np.testing.assert_allclose(transforms.dct2(N) @ x, sfft.dct(x, type=2) / 2, **tol)
    np.testing.assert_allclose(transforms.dst2(N) @ x, sfft.dst(x, type=2) / 2, **tol)
    np.testing.assert_allclose(transforms.dct3(N) @ x, sfft.dct(x, type=3) / 2, **tol)
    np.testing.assert_allclose(transforms.dst3(N) @ x, sfft.dst(x, type=3) / 2, **tol)


@pytest.mark.parametrize("N", SIZES)
@pytest.mark.parametrize("kind", "PND")
def test_inverse_pairs(N, kind):
    M = transforms.inverse_matrix(kind, N) @ transforms.forward_matrix(kind, N)
    np.testing.assert_allclose(M, np.eye(N), rtol=0, atol=1e-13 * max(1, N))


def test_hand_cases():
    # N = 1: every transform is the identity (cos 0 = 1, sin(pi/2) = 1); DCT-III halves u_0.
    assert transforms.dct2(1)[0, 0] == 1.0
    assert transforms.dst2(1)[0, 0] == 1.0
    assert transforms.dct3(1)[0, 0] == 0.5
    assert transforms.dst3(1)[0, 0] == 0.5
    # N = 2 by hand: DCT-II rows [1, 1], [cos(pi/4), cos(3 pi/4)]
    c = np.sqrt(0.5)
    np.testing.assert_allclose(transforms.dct2(2), [[1, 1], [c, -c]], atol=1e-15)
    # DST-II rows [sin(pi/4), sin(3pi/4)], [sin(pi/2), sin(3pi/2)]
    np.testing.assert_allclose(transforms.dst2(2), [[c, c], [1, -1]], atol=1e-15)
    # DFT of length 2
    np.testing.assert_allclose(transforms.dft(2), [[1, 1], [1, -1]], atol=1e-15)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 7, 8, 12, 32, 64])
@pytest.mark.parametrize("kind", "PND")
def test_eigen_invariant(N, kind):
    """A_1d phi_k = lam_k phi_k for the 1-D operator assembled from the ghost rules."""
    h = 0.37
    A = assemble_matrix((1, 1, N), kind * 2 + "PPPP", (h, 1.0, 1.0))  # y, z of size 1 periodic: zero
    lam = eigenvalues(kind, N, h)
    # eigenvectors: conjugate-transposed rows of the forward transform are the basis functions
    basis = np.conj(transforms.forward_matrix(kind, N))
    for k in range(N):
        phi = basis[k]
        np.testing.assert_allclose(A @ phi, lam[k] * phi, rtol=0, atol=1e-12 / h**2)


def test_eigenvalue_table_values():
    # Table eig at unit spacing, by hand: periodic n=4 -> 0, -2, -4, -2; Neumann n=2 -> 0, -2;
    # Dirichlet n=1 -> -4 (a single cell with both ghosts -u0).
    np.testing.assert_allclose(eigenvalues("P", 4, 1.0), [0, -2, -4, -2], atol=1e-15)
    np.testing.assert_allclose(eigenvalues("N", 2, 1.0), [0, -2], atol=1e-15)
    np.testing.assert_allclose(eigenvalues("D", 1, 1.0), [-4], atol=1e-15)
    np.testing.assert_allclose(eigenvalues("D", 2, 0.5), [-8, -16], atol=1e-13)
