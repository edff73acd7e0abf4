"""Reference oracle for the FFT + Thomas Poisson solve (PittPack, arXiv:1909.05423).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package: only ``tests/``, ``__graft_entry__.smoke``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP path (no kernels, tables, constants or helpers).

What it computes: the exact discrete solution ``u`` of the second-order 7-point
problem ``L_h u = f`` on a uniform cell-centred grid (section "Mathematical
Formulation", Eq. 3) with per-face periodic / homogeneous Dirichlet /
homogeneous Neumann conditions (section "Boundary Conditions"), written as the
paper's algorithm: forward transforms along x then y (Table
TransformationList), one tridiagonal solve along z per wavenumber pair using the
modified wavenumbers of Table eig (section "Solution of the Resulting
Tridiagonal Matrices", Algorithm Thomas), the inverse transforms, and the
zero-mode treatment of section "Well-posedness".

Plain float64 numpy throughout: transforms are explicit direct-sum matrices
applied as matrix products (no FFT, no blocking, no fusion); the tridiagonal
solves are the general Thomas algorithm vectorised over lines.

Modules
-------
transforms   direct-sum DFT / DCT-II / DCT-III / DST-II / DST-III matrices
eigen        1-D eigenvalues (Table eig)
thomas       general Thomas algorithm (Algorithm Thomas, read as standard)
operator     the assembled 7-point operator and its stencil application
solver       solve() and solve_adjoint()
dense        brute-force dense solves of the assembled matrix (tiny grids)
closed_form  exact discrete solutions for sums of discrete eigenmodes
"""

from .solver import solve, solve_adjoint, is_singular, parse_bc  # noqa: F401
from .operator import apply_laplacian, assemble_matrix, backward_error  # noqa: F401
