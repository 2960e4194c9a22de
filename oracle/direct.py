"""Exact discrete solution u = A^-1 b of the symmetric-form system (the
Green's matrix G = A^-1 of Section 2).  Parity pinned (dense LAPACK solve on
tiny grids and G = G^T; tests/test_oracle_operator.py)."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def solve(A, b):
    """Sparse LU (SuperLU) solve; b may hold several columns."""
    lu = spla.splu(sp.csc_matrix(A), permc_spec="MMD_AT_PLUS_A")
    return lu.solve(np.asarray(b, dtype=np.complex128))


def dense_inverse(A):
    """G = A^-1 as a dense matrix (tiny grids only)."""
    return np.linalg.inv(np.asarray(sp.csr_matrix(A).todense()))
