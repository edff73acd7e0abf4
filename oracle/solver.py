"""The oracle solve and its literal adjoint (test infrastructure; see package docstring).

Algorithm (the paper's order):
  1. singular case with projection: subtract the volume mean of f (section
     "Well-posedness", the alternative it names: integrate the source over the
     volume and subtract it);
  2. forward transform along x, then along y (Table TransformationList), as
     direct-sum matrix products;
  3. for every wavenumber pair (kx, ky) solve the z tridiagonal system
     (section "Solution of the Resulting Tridiagonal Matrices"):
         (u_{k-1} - 2 u_k + u_{k+1}) / hz^2 + (lam_x + lam_y) u_k = fhat_k
     with lam from Table eig and the z face rules folded into the end rows
     (Dirichlet: diagonal -3/hz^2 + lam, Neumann: -1/hz^2 + lam); periodic z is
     a cyclic system (Sherman-Morrison, mentioned in the Thomas subsection);
  4. the singular system (kx, ky) = (0, 0) of a pure Neumann/periodic problem is
     pinned: its first unknown is fixed to zero and the remaining rows are solved
     (the paper's default, "Well-posedness": the corner value, i.e. the mean of
     the solution over the first z plane, is kept fixed);
  5. inverse transforms along y, then x;
  6. gauge 'mean' only: subtract the volume mean of u (zero-mean gauge).

Gauges (only matter in the singular case):
  'mean'     project f, pin, then subtract mean(u)   -> unique zero-mean solution
  'pin'      project f, pin                          -> mean of u over plane z=0 is 0
  'pin_raw'  pin only (the paper's default, no projection)

solve_adjoint applies the literal transpose of every step of solve, in reverse
order, with the transposes taken of the same matrices (conjugate transposes for
the complex DFT steps) and of the same tridiagonal systems.
"""

import numpy as np

from . import transforms
from .eigen import eigenvalues
from .thomas import thomas, thomas_cyclic

GAUGES = ("mean", "pin", "pin_raw")


def parse_bc(bc):
    """Validate a 6-character boundary string (x-, x+, y-, y+, z-, z+)."""
    if not isinstance(bc, str) or len(bc) != 6 or any(ch not in "PDN" for ch in bc):
        raise ValueError(f"bc must be 6 characters from 'PDN', got {bc!r}")
    for d, name in ((0, "x"), (1, "y")):
        if bc[2 * d] != bc[2 * d + 1]:
            raise ValueError(f"both {name} faces must share a type (Table eig), got {bc!r}")
    if ("P" in bc[4:6]) and bc[4:6] != "PP":
        raise ValueError(f"periodic z needs both z faces periodic, got {bc!r}")
    return bc


def is_singular(bc):
    """True when the operator has the constant null vector: x, y in {P, N} and z pure N or P."""
    return bc[0] in "PN" and bc[2] in "PN" and bc[4:6] in ("NN", "PP")


def _z_coefficients(lam, nz, bc, hz):
    """Tridiagonal coefficients (a, b, c) of the z systems, shape lam.shape + (nz,)."""
    w = 1.0 / (hz * hz)
    shape = lam.shape + (nz,)
    a = np.full(shape, w)
    c = np.full(shape, w)
    b = np.broadcast_to((-2.0 * w + lam)[..., None], shape).copy()
    if bc[4:6] != "PP":
        for idx, kind in ((0, bc[4]), (nz - 1, bc[5])):
            b[..., idx] += -w if kind == "D" else w
        a[..., 0] = 0.0
        c[..., nz - 1] = 0.0
    return a, b, c


def _solve_lines(a, b, c, r, periodic, transpose):
    """Solve every z line (last axis); transpose=True solves with the transposed matrix."""
    if transpose:
        # (A^T)[i, i-1] = A[i-1, i] = c_{i-1};  (A^T)[i, i+1] = A[i+1, i] = a_{i+1}
        a, c = np.roll(c, 1, axis=-1), np.roll(a, -1, axis=-1)
    nz = r.shape[-1]
    if not periodic:
        return thomas(a, b, c, r)
    if nz >= 3:
        return thomas_cyclic(a, b, c, r)
    # one or two cells in a periodic direction: assemble each small system
    M = np.zeros(b.shape + (nz,))
    for i in range(nz):
        M[..., i, i] += b[..., i]
        M[..., i, (i - 1) % nz] += a[..., i]
        M[..., i, (i + 1) % nz] += c[..., i]
    return np.linalg.solve(M, r[..., None])[..., 0]


def _pinned_line(a, b, c, r, periodic, transpose):
    """The (0,0) system with its first unknown fixed to zero: solve rows/cols 1..nz-1."""
    x = np.zeros(r.shape, dtype=np.result_type(r, b))
    if r.shape[-1] > 1:
        aa, bb, cc = a[..., 1:].copy(), b[..., 1:], c[..., 1:].copy()
        aa[..., 0] = 0.0          # coupling to the pinned unknown (value zero)
        cc[..., -1] = 0.0         # periodic wrap to the pinned unknown (value zero)
        x[..., 1:] = _solve_lines(aa, bb, cc, r[..., 1:], False, transpose)
    return x


def _spectral_solve(fh, bc, h, shape, transpose):
    """Step 3-4 on spectral data fh of shape (..., nz, ny, nx) (complex or real)."""
    nz, ny, nx = shape
    lam = eigenvalues(bc[2], ny, h[1])[:, None] + eigenvalues(bc[0], nx, h[0])[None, :]
    a, b, c = _z_coefficients(lam, nz, bc, h[2])
    periodic = bc[4:6] == "PP"
    singular = is_singular(bc)
    if singular:
        b = b.copy()
        b[0, 0, :] = -3.0 / (h[2] * h[2])   # placeholder so the bulk solve stays finite
    r = np.ascontiguousarray(np.moveaxis(fh, -3, -1))   # (..., ny, nx, nz)
    x = _solve_lines(a, b, c, r, periodic, transpose)
    if singular:
        a0, b0, c0 = _z_coefficients(np.zeros(()), nz, bc, h[2])
        x[..., 0, 0, :] = _pinned_line(a0, b0, c0, r[..., 0, 0, :], periodic, transpose)
    return np.ascontiguousarray(np.moveaxis(x, -1, -3))


def _check(f, bc, h, gauge):
    parse_bc(bc)
    if gauge not in GAUGES:
        raise ValueError(f"gauge must be one of {GAUGES}, got {gauge!r}")
    f = np.asarray(f, dtype=np.float64)
    if f.ndim < 3:
        raise ValueError("f must have shape (..., nz, ny, nx)")
    if len(h) != 3 or any(not (hd > 0) for hd in h):
        raise ValueError("h must hold three positive spacings")
    return f


def _mean(v):
    return v.mean(axis=(-3, -2, -1), keepdims=True)


def solve(f, bc, h, gauge="mean", faces=None):
    """Exact discrete solution of L_h u = f (see module docstring); f: (..., nz, ny, nx).

    faces: optional non-homogeneous face values (see operator.py).  Their ghost
    contributions move to the right-hand side (Dirichlet subsection: "moved to
    the right hand side"), f <- f - L_h(0), and the homogeneous problem is solved.
    """
    f = _check(f, bc, h, gauge)
    nz, ny, nx = f.shape[-3:]
    if faces is not None:
        from .operator import boundary_lift
        for i, kind in enumerate(bc):
            if kind == "P" and faces[i] is not None:
                raise ValueError("periodic faces carry no values")
        f = f - boundary_lift(f.shape, bc, h, faces)
    singular = is_singular(bc)
    if singular and gauge in ("mean", "pin"):
        f = f - _mean(f)
    Xf = transforms.forward_matrix(bc[0], nx)
    Yf = transforms.forward_matrix(bc[2], ny)
    Xi = transforms.inverse_matrix(bc[0], nx)
    Yi = transforms.inverse_matrix(bc[2], ny)
    fh = f @ Xf.T                   # along x
    fh = np.matmul(Yf, fh)          # along y
    uh = _spectral_solve(fh, bc, h, (nz, ny, nx), transpose=False)
    u = np.matmul(Yi, uh)           # inverse along y
    u = u @ Xi.T                    # inverse along x
    u = np.real(u) if np.iscomplexobj(u) else u
    if singular and gauge == "mean":
        u = u - _mean(u)
    return np.ascontiguousarray(u)


def solve_adjoint(g, bc, h, gauge="mean"):
    """Transpose of solve() applied to g: every step transposed, in reverse order."""
    g = _check(g, bc, h, gauge)
    nz, ny, nx = g.shape[-3:]
    singular = is_singular(bc)
    if singular and gauge == "mean":
        g = g - _mean(g)            # transpose of the final demean (a symmetric projection)
    Xf = transforms.forward_matrix(bc[0], nx)
    Yf = transforms.forward_matrix(bc[2], ny)
    Xi = transforms.inverse_matrix(bc[0], nx)
    Yi = transforms.inverse_matrix(bc[2], ny)
    # transpose of "v -> v @ M.T" is "v -> v @ conj(M)"; of "v -> M @ v" is "v -> M^H @ v"
    gh = g.astype(np.complex128) if (bc[0] == "P" or bc[2] == "P") else g
    gh = gh @ np.conj(Xi)
    gh = np.matmul(np.conj(Yi).T, gh)
    vh = _spectral_solve(gh, bc, h, (nz, ny, nx), transpose=True)
    v = np.matmul(np.conj(Yf).T, vh)
    v = v @ np.conj(Xf)
    v = np.real(v) if np.iscomplexobj(v) else v
    if singular and gauge in ("mean", "pin"):
        v = v - _mean(v)            # transpose of the initial projection
    return np.ascontiguousarray(v)
