"""Auxiliary problems H^M_q, H^R_p, H^L_p, their LU factorizations and the
auxiliary Green's operators G~.  Parity pinned (dense inverse of the
assembled H, the bordered Dirichlet problem, and H^M_1 = A when m = 1;
tests/test_oracle_subproblem.py).

Section 3.1, "Auxiliary problems" and "Auxiliary Green's operators" (the same
text in Section 4.1 for 3D, Section 2.1 in 1D):

* H^M_q is the discretization on X^M_q of the Helmholtz problem whose sweep-axis
  PML vanishes on X_q, with zero Dirichlet data.  G~^M_q y: put y on X_q and 0 on
  the pads, solve, restrict to X_q.
* H^R_p is the discretization on X^R_p with Dirichlet data w on the line just
  left of X^R_p.  Moving that known value to the right-hand side of the first
  line gives g = (-coupling) * w, which is the paper's g = (-1/h^2)[w, 0, ...]
  (the coupling of the symmetric form is 1/(h^2 * prod of the cross-axis s),
  which equals 1/h^2 where the cross axes carry no PML).  G~^R_p w: solve,
  restrict to X_p.
* H^L_p: the same with the data on the line just right of X^L_p, g = [0, ..., -coupling*w].

Factorization (Algorithm 1 / Section 3.1): the 2D subproblems are quasi-1D; the
unknowns are reordered with the sweep axis fastest, which makes H banded with
bandwidth L (lines of the subproblem), and factored by banded LU (LAPACK
zgbtrf, partial pivoting).  In 3D (Algorithm 3) the paper applies nested
dissection to the reordered quasi-2D problem; here a sparse LU with a
fill-reducing column ordering (SuperLU, COLAMD) stands in for it: the factorization differs,
the operator it inverts does not.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.linalg import lapack

from .partition import Sub


def _widths(prob, sub):
    """PML widths of the sweep-axis profile below and above its zero region
    (the sub's own, or gamma on both sides for a Sub built without them)."""
    return (sub.gamma_lo or prob.gamma, sub.gamma_hi or prob.gamma)


class BandLU:
    """Banded LU of a sparse matrix (LAPACK zgbtrf / zgbtrs)."""

    def __init__(self, A, kl, ku):
        A = sp.coo_matrix(A)
        N = A.shape[0]
        ab = np.zeros((2 * kl + ku + 1, N), dtype=np.complex128)
        if np.any(A.row - A.col > kl) or np.any(A.col - A.row > ku):
            raise ValueError("matrix exceeds the stated bandwidth")
        ab[kl + ku + A.row - A.col, A.col] = A.data
        lu, piv, info = lapack.zgbtrf(ab, kl, ku)
        if info != 0:
            raise np.linalg.LinAlgError(f"zgbtrf info={info}")
        self.lu, self.piv, self.kl, self.ku = lu, piv, kl, ku

    def solve(self, rhs):
        x, info = lapack.zgbtrs(self.lu, self.kl, self.ku, rhs, self.piv)
        if info != 0:
            raise np.linalg.LinAlgError(f"zgbtrs info={info}")
        return x


class SparseLU:
    def __init__(self, A):
        self.lu = spla.splu(sp.csc_matrix(A), permc_spec="COLAMD")

    def solve(self, rhs):
        return self.lu.solve(rhs)


class Subproblem:
    """One auxiliary problem: operator, factorization and G~."""

    def __init__(self, prob, sub: Sub, X_p, factor=True):
        self.prob, self.sub = prob, sub
        self.X_p = X_p                 # (s_p, e_p) of the layer this G~ restricts to
        self.L = sub.L
        self.H = prob.box_operator(sub.lo, sub.hi, sub.phi, sub.psi, _widths(prob, sub))
        self.lu = None
        self._coupling = None
        if factor:
            self.factor()

    # -- Algorithm 1 / 3: factor H -------------------------------------------------
    def _sweep_fastest(self):
        """Permutation new -> old that makes the sweep axis the fastest index."""
        S, L = self.prob.S, self.L
        old = np.arange(S * L).reshape((L, S))     # old index = cross + S * line
        return old.T.reshape(-1)                   # new index = line + L * cross

    def factor(self):
        d = self.prob.d
        if d <= 2:
            perm = self._sweep_fastest()
            Hp = self.H[perm][:, perm]
            bw = self.L
            self.lu = BandLU(Hp, bw, bw)
            self.perm = perm
        else:
            self.lu = SparseLU(self.H)
            self.perm = None
        return self

    def solve(self, g):
        """v = H^-1 g for g on the subproblem grid (column-major)."""
        if self.lu is None:
            self.factor()
        if self.perm is None:
            return self.lu.solve(np.asarray(g, dtype=np.complex128))
        gp = np.asarray(g, dtype=np.complex128)[self.perm]
        v = np.empty_like(gp)
        v[self.perm] = self.lu.solve(gp)
        return v

    # -- index helpers ---------------------------------------------------------------
    def _slice_of_lines(self, a, b):
        S, lo = self.prob.S, self.sub.lo
        return slice((a - lo) * S, (b - lo + 1) * S)

    def restrict(self, v):
        return v[self._slice_of_lines(*self.X_p)]

    def boundary_coupling(self):
        """Coupling of the subproblem's first (R) or last (L) line to the Dirichlet
        line beyond it, read off the symmetric operator on the grid extended by
        that line (the discrete problem before the known value is moved to the
        right-hand side).  Returns the diagonal of that S x S block."""
        if self._coupling is not None:
            return self._coupling
        S, sub = self.prob.S, self.sub
        if sub.kind == "R":
            Hx = self.prob.box_operator(sub.lo - 1, sub.hi, sub.phi, sub.psi, _widths(self.prob, sub))
            blk = Hx[S:2 * S, 0:S]
        elif sub.kind == "L":
            Hx = self.prob.box_operator(sub.lo, sub.hi + 1, sub.phi, sub.psi, _widths(self.prob, sub))
            n_rows = Hx.shape[0]
            blk = Hx[n_rows - 2 * S:n_rows - S, n_rows - S:n_rows]
        else:
            raise ValueError("M subproblems have no Dirichlet data")
        blk = sp.csr_matrix(blk)
        diag = blk.diagonal()
        if abs(blk - sp.diags(diag)).sum() != 0:
            raise AssertionError("boundary coupling is not diagonal")
        self._coupling = diag
        return diag

    # -- auxiliary Green's operators ------------------------------------------------------
    def G(self, data):
        """G~^M y (data = y on X_q), G~^R w or G~^L w (data = w on one line)."""
        S, sub = self.prob.S, self.sub
        g = np.zeros(S * self.L, dtype=np.complex128)
        if sub.kind == "M":
            g[self._slice_of_lines(*self.X_p)] = data
        elif sub.kind == "R":
            g[0:S] = -self.boundary_coupling() * data
        else:
            g[S * (self.L - 1):] = -self.boundary_coupling() * data
        return self.restrict(self.solve(g))
