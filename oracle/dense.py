"""Brute-force solves of the assembled 7-point matrix (test infrastructure).

Used on tiny grids (at most a few hundred unknowns) to pin the transform-based
oracle to the plain definition of the discrete problem: the matrix A comes from
operator.assemble_matrix (the stencil of Eq. 3 with the ghost rules) and is
solved with a dense LU (numpy.linalg.solve).

Singular case (constant null vector, section "Well-posedness"):
  'mean'     bordered system [[A, 1], [1^T, 0]] [u; c] = [f; 0]:
             A u = f - c 1 (c = mean f, the projection) and sum(u) = 0.
  'pin'      the 'mean' solution shifted so that its mean over the plane z = 0 is 0.
  'pin_raw'  bordered system [[A, -e], [e^T, 0]] [u; c] = [f; 0] with e the
             indicator of the plane z = 0: every equation holds except that the
             plane-0 rows absorb a common constant, and the plane-0 sum of u is 0.
"""

import numpy as np

from .operator import assemble_matrix
from .solver import is_singular, parse_bc


def dense_solve(f, bc, h, gauge="mean"):
    parse_bc(bc)
    f = np.asarray(f, dtype=np.float64)
    nz, ny, nx = f.shape
    n = f.size
    A = assemble_matrix((nz, ny, nx), bc, h)
    rhs = f.reshape(-1)
    if not is_singular(bc):
        return np.linalg.solve(A, rhs).reshape(f.shape)
    plane0 = np.zeros(n)
    plane0[: nx * ny] = 1.0
    if gauge in ("mean", "pin"):
        border = np.ones(n)
        M = np.block([[A, border[:, None]], [border[None, :], np.zeros((1, 1))]])
        u = np.linalg.solve(M, np.concatenate([rhs, [0.0]]))[:n].reshape(f.shape)
        if gauge == "pin":
            u = u - u[0].mean()
        return u
    if gauge == "pin_raw":
        M = np.block([[A, -plane0[:, None]], [plane0[None, :], np.zeros((1, 1))]])
        return np.linalg.solve(M, np.concatenate([rhs, [0.0]]))[:n].reshape(f.shape)
    raise ValueError(f"unknown gauge {gauge!r}")


def dense_operator(shape, bc, h, gauge="mean"):
    """The solve as an explicit n x n matrix G (columns = responses to unit sources)."""
    nz, ny, nx = shape
    n = nz * ny * nx
    G = np.empty((n, n))
    for q in range(n):
        e = np.zeros(n)
        e[q] = 1.0
        G[:, q] = dense_solve(e.reshape(shape), bc, h, gauge).reshape(-1)
    return G
