"""General Thomas algorithm (section "Thomas Algorithm", Algorithm Thomas).

Test infrastructure; see the package docstring.

The printed algorithm carries typesetting errors (an undefined ``bet``, a
doubled ``r`` in the forward update and a flipped sign in back substitution).
Reading used here is the standard algorithm the section describes:

    forward:   aux_0 = b_0,               g_0 = c_0 / aux_0,   r_0 = r_0 / aux_0
               aux_i = b_i - a_i g_{i-1},  g_i = c_i / aux_i,   r_i = (r_i - a_i r_{i-1}) / aux_i
    backward:  x_{N-1} = r_{N-1},          x_i = r_i - g_i x_{i+1}

with a_i the sub-diagonal (a_0 unused), b_i the diagonal and c_i the
super-diagonal (c_{N-1} unused).  No pivoting: the systems met here are
diagonally dominant (the singular zero mode is handled by the caller).

The arrays may carry leading batch axes; the recurrence runs along the last
axis and is vectorised over the others (one system per batch index).  The
periodic variant uses the Sherman-Morrison splitting the same section mentions
for periodic z.
"""

import numpy as np


def thomas(a, b, c, r):
    """Solve the tridiagonal systems (a, b, c) x = r along the last axis.

    a, b, c broadcast against r; r may be real or complex.  Returns x with the
    dtype of r promoted with the coefficients.
    """
    r = np.asarray(r)
    shape = np.broadcast_shapes(np.shape(a), np.shape(b), np.shape(c), r.shape)
    a = np.broadcast_to(a, shape)
    b = np.broadcast_to(b, shape)
    c = np.broadcast_to(c, shape)
    dtype = np.result_type(a, b, c, r)
    r = np.broadcast_to(r, shape)
    n = shape[-1]
    g = np.empty(shape, dtype=np.result_type(a, b, c))
    x = np.empty(shape, dtype=dtype)
    aux = b[..., 0]
    g[..., 0] = c[..., 0] / aux
    x[..., 0] = r[..., 0] / aux
    for i in range(1, n):
        aux = b[..., i] - a[..., i] * g[..., i - 1]
        g[..., i] = c[..., i] / aux
        x[..., i] = (r[..., i] - a[..., i] * x[..., i - 1]) / aux
    for i in range(n - 2, -1, -1):
        x[..., i] = x[..., i] - g[..., i] * x[..., i + 1]
    return x


def thomas_cyclic(a, b, c, r):
    """Solve cyclic tridiagonal systems: row 0 couples to x_{N-1} through a_0 and
    row N-1 couples to x_0 through c_{N-1}.  Sherman-Morrison splitting into two
    ordinary Thomas solves (requires N >= 3)."""
    r = np.asarray(r)
    shape = np.broadcast_shapes(np.shape(a), np.shape(b), np.shape(c), r.shape)
    a = np.broadcast_to(a, shape)
    b = np.array(np.broadcast_to(b, shape), dtype=np.result_type(a, b, c))
    c = np.broadcast_to(c, shape)
    alpha = c[..., -1]          # A[N-1, 0]
    beta = a[..., 0]            # A[0, N-1]
    gamma = -b[..., 0]
    bb = b.copy()
    bb[..., 0] = b[..., 0] - gamma
    bb[..., -1] = b[..., -1] - alpha * beta / gamma
    aa = np.array(a)
    aa[..., 0] = 0.0
    cc = np.array(c)
    cc[..., -1] = 0.0
    y = thomas(aa, bb, cc, r)
    uvec = np.zeros(shape, dtype=bb.dtype)
    uvec[..., 0] = gamma
    uvec[..., -1] = alpha
    z = thomas(aa, bb, cc, uvec)
    # v = (1, 0, ..., 0, beta / gamma)
    vy = y[..., 0] + (beta / gamma) * y[..., -1]
    vz = z[..., 0] + (beta / gamma) * z[..., -1]
    fact = vy / (1.0 + vz)
    return y - fact[..., None] * z
