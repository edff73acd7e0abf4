"""MI355X-native FFT + Thomas Poisson solver (PittPack's hot path, arXiv:1909.05423).

The solve runs in hand-written HIP kernels behind the C ABI of
include/ppsolve.h (libppsolve.so, built in-tree); this package is the thin
Python binding on top of it.
"""

from .solver import Plan, PoissonSolve, poisson_solve  # noqa: F401
