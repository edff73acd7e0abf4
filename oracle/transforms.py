"""Direct-sum transform matrices (test infrastructure; see package docstring).

Each function returns the dense N x N matrix of one transform exactly as the
paper defines it in section "Boundary Conditions"; a transform of a vector v is
``M @ v``.  Angles are reduced exactly over the integers before the single
floating-point multiply by pi, so every entry is cos/sin of an angle in
[0, 2*pi) that carries one rounding.

Definitions (index k = output, n = input):

* DFT, periodic faces (Eq. for the periodic condition):
      Y_k = sum_n u_n exp(-2 pi i k n / N)
* DCT-II ("DCT10"), Neumann forward (Neumann subsection):
      Y_k = sum_n u_n cos((n + 1/2) k pi / N)
* DCT-III ("DCT01"), Neumann inverse (Neumann subsection):
      Y_k = u_0 / 2 + sum_{n>=1} u_n cos((k + 1/2) n pi / N)
* DST-II ("DST10"), Dirichlet forward (Dirichlet subsection):
      Y_k = sum_n u_n sin((n + 1/2)(k + 1) pi / N)
* DST-III ("DST01"), Dirichlet inverse.  The printed formula in the Dirichlet
  subsection is garbled (a cosine, mixed indices).  Reading used here: the
  transform that inverts DST-II up to 2/N, i.e.
      Y_n = (-1)^n u_{N-1} / 2 + sum_{k=0}^{N-2} u_k sin((k + 1) (n + 1/2) pi / N)
  which is the matrix transpose of DST-II with weight 1/2 on its last column.

Exact inverses (checked in the tests): IDFT = conj(DFT)/N,
(2/N) DCT-III DCT-II = I, (2/N) DST-III DST-II = I.
"""

import numpy as np


def _cos_pi(num, den):
    """cos(pi * num / den) for integer arrays, with num reduced mod 2*den first."""
    num = np.mod(np.asarray(num, dtype=np.int64), 2 * den)
    return np.cos(np.pi * (num.astype(np.float64) / den))


def _sin_pi(num, den):
    """sin(pi * num / den) for integer arrays, with num reduced mod 2*den first."""
    num = np.mod(np.asarray(num, dtype=np.int64), 2 * den)
    return np.sin(np.pi * (num.astype(np.float64) / den))


def dft(N):
    """Forward DFT matrix F[k, n] = exp(-2 pi i k n / N)."""
    k = np.arange(N)[:, None]
    n = np.arange(N)[None, :]
    p = 2 * k * n
    return _cos_pi(p, N) - 1j * _sin_pi(p, N)


def idft(N):
    """Exact inverse of dft(N): conj(F) / N."""
    return np.conj(dft(N)) / N


def dct2(N):
    """DCT-II (the paper's DCT10), C2[k, n] = cos(pi (2n+1) k / (2N))."""
    k = np.arange(N)[:, None]
    n = np.arange(N)[None, :]
    return _cos_pi((2 * n + 1) * k, 2 * N)


def dct3(N):
    """DCT-III (the paper's DCT01), C3[k, n] = w_n cos(pi (2k+1) n / (2N)), w_0 = 1/2."""
    k = np.arange(N)[:, None]
    n = np.arange(N)[None, :]
    m = _cos_pi((2 * k + 1) * n, 2 * N)
    m[:, 0] *= 0.5
    return m


def dst2(N):
    """DST-II (the paper's DST10), S2[k, n] = sin(pi (2n+1)(k+1) / (2N))."""
    k = np.arange(N)[:, None]
    n = np.arange(N)[None, :]
    return _sin_pi((2 * n + 1) * (k + 1), 2 * N)


def dst3(N):
    """DST-III (the paper's DST01, corrected reading), S3[n, k] = w_k sin(pi (k+1)(2n+1) / (2N)),
    w_{N-1} = 1/2."""
    n = np.arange(N)[:, None]
    k = np.arange(N)[None, :]
    m = _sin_pi((k + 1) * (2 * n + 1), 2 * N)
    m[:, N - 1] *= 0.5
    return m


def forward_matrix(kind, N):
    """Forward transform for one direction (Table TransformationList):
    'P' -> DFT, 'N' -> DCT-II, 'D' -> DST-II."""
    if kind == "P":
        return dft(N)
    if kind == "N":
        return dct2(N)
    if kind == "D":
        return dst2(N)
    raise ValueError(f"unknown boundary type {kind!r}")


def inverse_matrix(kind, N):
    """Exact inverse of forward_matrix(kind, N) (Table TransformationList):
    'P' -> IDFT, 'N' -> (2/N) DCT-III, 'D' -> (2/N) DST-III."""
    if kind == "P":
        return idft(N)
    if kind == "N":
        return (2.0 / N) * dct3(N)
    if kind == "D":
        return (2.0 / N) * dst3(N)
    raise ValueError(f"unknown boundary type {kind!r}")
