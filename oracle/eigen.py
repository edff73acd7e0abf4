"""One-dimensional eigenvalues of the second-difference operator (Table eig).

Test infrastructure; see the package docstring.

Table eig lists, for mode k of a direction with n cells:

    periodic              -2 + 2 cos(2 k pi / n)
    Neumann-Neumann       -2 + 2 cos(k pi / n)
    Dirichlet-Dirichlet   -2 + 2 cos((k + 1) pi / n)

for unit spacing; with spacing h each is divided by h^2 (the stencil of Eq. 3
divides by the squared spacing).  Section "Eigenvalues" adds the eigenvalues of
the directions to obtain the multi-dimensional one.
"""

import numpy as np


def eigenvalues(kind, n, h):
    """Return the length-n array of eigenvalues for boundary type kind in {'P','N','D'}."""
    k = np.arange(n, dtype=np.int64)
    if kind == "P":
        num, den = 2 * k, n
    elif kind == "N":
        num, den = k, n
    elif kind == "D":
        num, den = k + 1, n
    else:
        raise ValueError(f"unknown boundary type {kind!r}")
    num = np.mod(num, 2 * den)
    # -2 + 2 cos(t) evaluated as -4 sin^2(t / 2): the same value without the
    # cancellation that costs -2 + 2 cos(t) its relative accuracy for small t.
    half_angle = 0.5 * np.pi * (num.astype(np.float64) / den)
    return -4.0 * np.sin(half_angle) ** 2 / (h * h)
