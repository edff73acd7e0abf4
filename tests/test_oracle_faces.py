"""Pins of the oracle with non-homogeneous face values (Dirichlet values g on
the face, Neumann outward normal derivatives g; section "Boundary Conditions",
where the ghost values' known parts move to the right-hand side).

* Multilinear harmonic fields are reproduced exactly: the linear ghost
  extrapolation is exact for fields linear in the face normal, and the 3-point
  second difference of a linear function is zero.  A dropped factor 2 in the
  Dirichlet lift, a wrong sign of a Neumann derivative or a face put on the
  wrong side all fail this.
* The lift itself against an independent loop over the boundary cells, and the
  solve with faces against dense LU of the assembled matrix with that lift.
* Second-order convergence to a smooth solution with non-zero boundary data.
"""

import itertools

import numpy as np
import pytest

import oracle
from oracle import solver
from oracle.dense import dense_solve
from oracle.operator import apply_laplacian, boundary_lift


def _centres(shape, h):
    nz, ny, nx = shape
    x = (np.arange(nx) + 0.5) * h[0]
    y = (np.arange(ny) + 0.5) * h[1]
    z = (np.arange(nz) + 0.5) * h[2]
    return np.meshgrid(z, y, x, indexing="ij")   # Z, Y, X with shape (nz, ny, nx)


def _face_values(bc, shape, h, u, grad):
    """Face data of the field u(x, y, z) with gradient grad(x, y, z) -> (ux, uy, uz):
    Dirichlet faces carry u on the face, Neumann faces the outward normal
    derivative; periodic faces carry nothing."""
    nz, ny, nx = shape
    L = (nx * h[0], ny * h[1], nz * h[2])
    x = (np.arange(nx) + 0.5) * h[0]
    y = (np.arange(ny) + 0.5) * h[1]
    z = (np.arange(nz) + 0.5) * h[2]
    faces = []
    for d in range(3):
        for side in range(2):
            kind = bc[2 * d + side]
            if kind == "P":
                faces.append(None)
                continue
            pos = 0.0 if side == 0 else L[d]
            if d == 0:
                Z, Y = np.meshgrid(z, y, indexing="ij")
                pt = (np.full_like(Z, pos), Y, Z)
            elif d == 1:
                Z, X = np.meshgrid(z, x, indexing="ij")
                pt = (X, np.full_like(Z, pos), Z)
            else:
                Y, X = np.meshgrid(y, x, indexing="ij")
                pt = (X, Y, np.full_like(Y, pos))
            if kind == "D":
                faces.append(u(*pt))
            else:
                n = -1.0 if side == 0 else 1.0
                faces.append(n * grad(*pt)[d])
    return faces


def _multilinear(bc, rng):
    """A random multilinear field constant along the periodic directions."""
    c = rng.standard_normal(8)
    vary = [bc[2 * d] != "P" for d in range(3)]
    terms = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (0, 1, 1), (1, 0, 1), (1, 1, 1)]
    coef = [ci if all(vary[d] or not e[d] for d in range(3)) else 0.0 for ci, e in zip(c, terms)]

    def u(x, y, z):
        return sum(ci * x ** e[0] * y ** e[1] * z ** e[2] for ci, e in zip(coef, terms))

    def grad(x, y, z):
        gx = sum(ci * e[0] * y ** e[1] * z ** e[2] for ci, e in zip(coef, terms) if e[0])
        gy = sum(ci * e[1] * x ** e[0] * z ** e[2] for ci, e in zip(coef, terms) if e[1])
        gz = sum(ci * e[2] * x ** e[0] * y ** e[1] for ci, e in zip(coef, terms) if e[2])
        zero = 0.0 * x
        return (gx + zero, gy + zero, gz + zero)

    return u, grad


FACE_BCS = [x + x + y + y + z for x in "PND" for y in "PND" for z in ("DD", "NN", "DN", "ND")]


@pytest.mark.parametrize("bc", FACE_BCS)
def test_multilinear_fields_reproduced_exactly(bc):
    rng = np.random.default_rng(sum(map(ord, bc)))
    for shape in [(4, 5, 6), (3, 7, 2), (6, 2, 5)]:
        h = tuple(rng.uniform(0.4, 1.5, 3))
        u, grad = _multilinear(bc, rng)
        Z, Y, X = _centres(shape, h)
        ustar = u(X, Y, Z) + 0.0 * X
        faces = _face_values(bc, shape, h, u, grad)
        # the operator with these faces annihilates the field
        r = apply_laplacian(ustar, bc, h, faces)
        scale = sum(4.0 / hd ** 2 for hd in h) * np.abs(ustar).max()
        assert np.abs(r).max() < 1e-12 * scale
        # and the solve with a zero source returns it (up to a constant when singular)
        uh = oracle.solve(np.zeros(shape), bc, h, "mean", faces=faces)
        if solver.is_singular(bc):
            uh, ustar = uh - uh.mean(), ustar - ustar.mean()
        assert np.abs(uh - ustar).max() < 1e-11 * max(1.0, np.abs(ustar).max()), bc


def _lift_by_cells(shape, bc, h, faces):
    """L_h(0) with face values, cell by cell from the ghost rules: a Dirichlet
    ghost 2g - u_b contributes 2g/h^2 to its boundary cell, a Neumann ghost
    u_b + h g contributes g/h."""
    nz, ny, nx = shape
    out = np.zeros(shape)
    n = (nx, ny, nz)
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        idx = (i, j, k)
        for d in range(3):
            for side in range(2):
                kind = bc[2 * d + side]
                at_face = idx[d] == (0 if side == 0 else n[d] - 1)
                if kind == "P" or not at_face or faces[2 * d + side] is None:
                    continue
                if d == 0:
                    g = faces[2 * d + side][k, j]
                elif d == 1:
                    g = faces[2 * d + side][k, i]
                else:
                    g = faces[2 * d + side][j, i]
                out[k, j, i] += 2.0 * g / h[d] ** 2 if kind == "D" else g / h[d]
    return out


@pytest.mark.parametrize("bc", ["DDNNDN", "NNDDND", "PPDDNN", "NNNNNN", "DDDDDD", "PPNNDD", "NNPPNN"])
def test_lift_and_solve_against_dense(bc):
    rng = np.random.default_rng(3 + sum(map(ord, bc)))
    for shape in [(3, 4, 5), (2, 3, 2), (5, 2, 4), (1, 1, 3)]:
        nz, ny, nx = shape
        h = tuple(rng.uniform(0.4, 1.5, 3))
        dims = [(nz, ny)] * 2 + [(nz, nx)] * 2 + [(ny, nx)] * 2
        faces = [None if bc[i] == "P" else rng.standard_normal(dims[i]) for i in range(6)]
        lift = _lift_by_cells(shape, bc, h, faces)
        np.testing.assert_allclose(boundary_lift(shape, bc, h, faces), lift, rtol=0, atol=1e-13 * np.abs(lift).max())
        f = rng.standard_normal(shape)
        for gauge in ["mean", "pin", "pin_raw"] if solver.is_singular(bc) else ["mean"]:
            u = oracle.solve(f, bc, h, gauge, faces=faces)
            ud = dense_solve(f - lift, bc, h, gauge)
            assert np.abs(u - ud).max() < 1e-12 * np.abs(ud).max(), (bc, shape, gauge)


@pytest.mark.parametrize("bc", ["DDNNDN", "NNDDND", "PPDDNN", "DDPPDD"])
def test_second_order_with_boundary_data(bc):
    """Smooth solution on the unit cube with non-zero face values and fluxes:
    the RMS error against the continuous solution falls by 4x per halving of h."""
    kx = 2 * np.pi if bc[0] == "P" else 1.3
    ky = 2 * np.pi if bc[2] == "P" else 0.9
    kz = 0.7

    def u(x, y, z):
        return np.cos(kx * x + 0.4) * np.sin(ky * y + 0.3) * np.cosh(kz * z) + 0.5

    def grad(x, y, z):
        return (-kx * np.sin(kx * x + 0.4) * np.sin(ky * y + 0.3) * np.cosh(kz * z),
                ky * np.cos(kx * x + 0.4) * np.cos(ky * y + 0.3) * np.cosh(kz * z),
                kz * np.cos(kx * x + 0.4) * np.sin(ky * y + 0.3) * np.sinh(kz * z))

    errs = []
    for n in (16, 32, 64):
        shape, h = (n, n, n), (1.0 / n,) * 3
        Z, Y, X = _centres(shape, h)
        f = (kz * kz - kx * kx - ky * ky) * (u(X, Y, Z) - 0.5)
        faces = _face_values(bc, shape, h, u, grad)
        uh = oracle.solve(f, bc, h, "mean", faces=faces)
        ustar = u(X, Y, Z)
        if solver.is_singular(bc):
            uh, ustar = uh - uh.mean(), ustar - ustar.mean()
        errs.append(np.sqrt(np.mean((uh - ustar) ** 2)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 2.0) < 0.1), (errs, orders)
