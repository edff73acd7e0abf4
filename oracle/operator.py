"""The discrete operator itself: 7-point stencil with ghost-cell boundary rules.

Test infrastructure; see the package docstring.

Grid: cell-centred and directionally uniform (section "Mathematical
Formulation", Eq. 3, and the figure of cell centres with the boundary on the
faces).  Arrays are C-ordered (..., nz, ny, nx): x is the last axis.

Stencil (Eq. 3):  sum_d (u_{+1} - 2 u + u_{-1}) / h_d^2 = f.

Ghost rules at a face (section "Boundary Conditions"):
  'P'  periodic: the ghost is the cell at the opposite end of the line.
  'D'  Dirichlet, value g on the face: the ghost follows from linear
       extrapolation through the face (Dirichlet subsection),
       u_ghost = 2 g - u_boundary_cell  (homogeneous: g = 0).
  'N'  Neumann, outward normal derivative g on the face:
       u_ghost = u_boundary_cell + h g  (homogeneous: g = 0, zero flux).

Face values, when given, are a sequence of six arrays (or None for zero) in
the face order (x-, x+, y-, y+, z-, z+): x faces have shape (..., nz, ny),
y faces (..., nz, nx), z faces (..., ny, nx).
"""

import numpy as np


def _ghost(cell, kind, opposite, value=None, h=None):
    if kind == "P":
        return opposite
    if kind == "D":
        return -cell if value is None else 2.0 * value - cell
    if kind == "N":
        return cell if value is None else cell + h * value
    raise ValueError(f"unknown boundary type {kind!r}")


def _face(faces, i, axis):
    """Face array i expanded with a unit axis in the position of its normal."""
    if faces is None or faces[i] is None:
        return None
    return np.expand_dims(np.asarray(faces[i], dtype=np.float64), axis)


def apply_laplacian(u, bc, h, faces=None):
    """Apply L_h (Eq. 3 with the ghost rules) to u of shape (..., nz, ny, nx).

    bc is a 6-character string (x-, x+, y-, y+, z-, z+); h = (hx, hy, hz);
    faces (optional) holds the face values of non-homogeneous D/N faces.
    """
    u = np.asarray(u)
    out = np.zeros_like(u)
    for d in range(3):                       # d = 0 -> x, 1 -> y, 2 -> z
        axis = u.ndim - 1 - d
        lo_kind, hi_kind = bc[2 * d], bc[2 * d + 1]
        first = np.take(u, [0], axis=axis)
        last = np.take(u, [u.shape[axis] - 1], axis=axis)
        g_lo = _ghost(first, lo_kind, last, _face(faces, 2 * d, axis), h[d])
        g_hi = _ghost(last, hi_kind, first, _face(faces, 2 * d + 1, axis), h[d])
        padded = np.concatenate([g_lo, u, g_hi], axis=axis)
        n = u.shape[axis]
        up = np.take(padded, np.arange(2, n + 2), axis=axis)
        dn = np.take(padded, np.arange(0, n), axis=axis)
        out = out + (up - 2.0 * u + dn) / (h[d] * h[d])
    return out


def assemble_matrix(shape, bc, h):
    """Dense matrix of L_h, assembled point by point from the stencil.

    shape = (nz, ny, nx); unknown index p = (k * ny + j) * nx + i.
    Each of the six neighbours contributes 1/h^2 to its column; a neighbour
    outside the grid is a ghost and is folded in by its rule (periodic: the
    wrapped cell; Dirichlet: -1 on the diagonal; Neumann: +1 on the diagonal).
    Intended for tiny grids (used by the brute-force checks).
    """
    nz, ny, nx = shape
    dims = (nx, ny, nz)
    n = nx * ny * nz
    A = np.zeros((n, n))

    def index(i, j, k):
        return (k * ny + j) * nx + i

    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                p = index(i, j, k)
                pos = [i, j, k]
                for d in range(3):
                    w = 1.0 / (h[d] * h[d])
                    A[p, p] -= 2.0 * w
                    for step, kind in ((-1, bc[2 * d]), (+1, bc[2 * d + 1])):
                        q = list(pos)
                        q[d] += step
                        if 0 <= q[d] < dims[d]:
                            A[p, index(*q)] += w
                        elif kind == "P":
                            q[d] %= dims[d]
                            A[p, index(*q)] += w
                        elif kind == "D":
                            A[p, p] -= w
                        elif kind == "N":
                            A[p, p] += w
                        else:
                            raise ValueError(f"unknown boundary type {kind!r}")
    return A


def operator_inf_norm(h):
    """Upper bound of ||L_h||_inf used by the backward error: sum_d 4 / h_d^2."""
    return sum(4.0 / (hd * hd) for hd in h)


def boundary_lift(shape, bc, h, faces):
    """The affine part of L_h under non-homogeneous faces: L_h(0) with the given
    face values (non-zero only in boundary cells).  L_h u = A u + lift, so the
    face values move to the right-hand side as f - lift."""
    return apply_laplacian(np.zeros(shape), bc, h, faces)


def backward_error(f, u, bc, h, faces=None):
    """Normwise backward error  ||f - L_h u||_inf / (||L_h||_inf ||u||_inf + ||f||_inf).

    Pass the right-hand side the solution was meant to satisfy (in the singular
    case with projection, the projected source).
    """
    r = np.asarray(f) - apply_laplacian(u, bc, h, faces)
    den = operator_inf_norm(h) * np.max(np.abs(u)) + np.max(np.abs(f))
    return float(np.max(np.abs(r)) / den) if den > 0 else 0.0
