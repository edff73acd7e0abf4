"""Exact discrete solutions for sources built from discrete eigenmodes.

Test infrastructure; see the package docstring.

For a one-dimensional factor cos(w x + phi) sampled at cell centres
x_i = (i + 1/2) h, the second difference of Eq. 3 gives

    (g(x+h) - 2 g(x) + g(x-h)) / h^2 = -(4 / h^2) sin^2(w h / 2) g(x)

in the interior; at a face the ghost rule (periodic / Dirichlet by linear
extrapolation / Neumann) reproduces the same identity when w matches the
boundary type (periodic: w = 2 pi m / L; Neumann: cos(m pi x / L);
Dirichlet: sin(m pi x / L)).  A product of such factors, or a plane wave
cos(wx x + wy y + phi) times a z factor (a sum of two such products with the
same eigenvalue), is therefore an eigenvector of L_h with eigenvalue

    Lambda = -sum_d (4 / h_d^2) sin^2(w_d h_d / 2),

and L_h u = sum_m a_m v_m is solved exactly by u = sum_m (a_m / Lambda_m) v_m.
With the continuous source f = -|w|^2 u* of a single product u* (the paper's
manufactured solutions, section "Order of Accuracy") this gives the discrete
solution u_h = u* |w|^2 / (-Lambda).
"""

import numpy as np


def cell_centres(n, length):
    h = length / n
    return (np.arange(n) + 0.5) * h


def eigenvalue(omegas, h):
    """Lambda for frequencies (wx, wy, wz) on spacings (hx, hy, hz)."""
    return -sum((4.0 / (hd * hd)) * np.sin(0.5 * w * hd) ** 2 for w, hd in zip(omegas, h))


def mode_values(mode, shape, lengths):
    """Evaluate one mode on the grid (nz, ny, nx).

    mode = dict(form='sep',    w=(wx, wy, wz), phase=(px, py, pz))
           -> cos(wx x + px) cos(wy y + py) cos(wz z + pz)
         | dict(form='xywave', w=(wx, wy, wz), phase=(pxy, pz))
           -> cos(wx x + wy y + pxy) cos(wz z + pz)
    """
    nz, ny, nx = shape
    x = cell_centres(nx, lengths[0])
    y = cell_centres(ny, lengths[1])
    z = cell_centres(nz, lengths[2])
    wx, wy, wz = mode["w"]
    if mode["form"] == "sep":
        px, py, pz = mode["phase"]
        xy = np.cos(wy * y + py)[:, None] * np.cos(wx * x + px)[None, :]
    elif mode["form"] == "xywave":
        pxy, pz = mode["phase"]
        xy = np.cos(wx * x[None, :] + wy * y[:, None] + pxy)
    else:
        raise ValueError(f"unknown mode form {mode['form']!r}")
    return np.cos(wz * z + pz)[:, None, None] * xy[None, :, :]


def mode_sum(modes, amplitudes, shape, lengths):
    out = np.zeros(shape)
    for mode, a in zip(modes, amplitudes):
        out += a * mode_values(mode, shape, lengths)
    return out


def solve_mode_sum(modes, amplitudes, shape, lengths):
    """Exact discrete solution of L_h u = sum_m a_m v_m (all v_m eigenvectors)."""
    h = tuple(L / n for L, n in zip(lengths, (shape[2], shape[1], shape[0])))
    coef = [a / eigenvalue(m["w"], h) for m, a in zip(modes, amplitudes)]
    return mode_sum(modes, coef, shape, lengths)


def solve_mode_sum_at(modes, amplitudes, shape, lengths, points):
    """The same exact solution evaluated only at the given (k, j, i) index triples."""
    nz, ny, nx = shape
    h = (lengths[0] / nx, lengths[1] / ny, lengths[2] / nz)
    pts = np.asarray(points)
    z = (pts[:, 0] + 0.5) * h[2]
    y = (pts[:, 1] + 0.5) * h[1]
    x = (pts[:, 2] + 0.5) * h[0]
    out = np.zeros(len(pts))
    for m, a in zip(modes, amplitudes):
        wx, wy, wz = m["w"]
        if m["form"] == "sep":
            px, py, pz = m["phase"]
            v = np.cos(wx * x + px) * np.cos(wy * y + py) * np.cos(wz * z + pz)
        else:
            pxy, pz = m["phase"]
            v = np.cos(wx * x + wy * y + pxy) * np.cos(wz * z + pz)
        out += (a / eigenvalue(m["w"], h)) * v
    return out


def manufactured_ratio(omegas, h):
    """u_h / u* for the source f = -|w|^2 u* of a single eigen-product u*."""
    w2 = sum(w * w for w in omegas)
    return w2 / (-eigenvalue(omegas, h))
