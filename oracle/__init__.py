"""FP64 CPU oracle for the parallel orbital-updating method (arXiv 1510.07230).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The HIP library never
calls it and shares no code, header, table or constant generator with it.

The oracle is deliberately plain: NumPy arrays in float64, library FFT / QR /
eigh used as single steps, no blocking, fusion or reordering.  Each function
names the passage of the paper it follows:

  ks.py     the discrete Kohn-Sham energy (section 2.1, eq. "energy"), the
            Hamiltonian H(rho) (section 2.1), the periodic Hartree and ionic
            potentials, LDA exchange, the exact discrete gradient and the
            forces at fixed orbitals.
  orth.py   Orth(.) of Algorithm B step 5: the unique QR factor with a positive
            diagonal of R (section 3.2 uses QR through Cholesky; both give the
            same factor in exact arithmetic).
  algm.py   Algorithm M (section 3.3) with n_org = 1 and subspace
            diagonalisation switched off: search direction z_i (section 3.2),
            Barzilai-Borwein step, non-monotone backtracking (eq. "ene-de").
  dense.py  brute-force checks on tiny grids: the dense Hamiltonian matrix,
            its eigenvalues, and a dense self-consistent-field solve.
  cg.py     an independent conjugate-gradient Poisson solver, used only to
            pin the FFT Poisson solve of ks.py.

Parity status of each function is listed in the docstring of the module that
defines it.  Every function here is pinned by a CPU test in tests/ (see the
test module names starting with test_oracle_).
"""
from . import ks, orth, algm, dense, cg  # noqa: F401
