"""Recursive sweeping of the 3D auxiliary problems (Section 5, last
direction): each quasi-2D auxiliary problem H of Algorithm 3 is itself solved
approximately by the additive sweeping preconditioner along x2, instead of
being factored exactly.  Parity pinned (one inner layer gives the exact G~;
the slab reordering reproduces H exactly; the inner apply equals its O(m^2)
form; the outer GMRES iteration counts at the 3D experiments' settings;
tests/test_oracle_recursive.py).

The auxiliary problem of lines lo..hi along x3 lives on the slab
(i1, i2, i3) in [1, n] x [1, n] x [lo, hi].  Taking x2 as its sweep axis
("sweeping along the x2 direction with the same technique") means the same
construction one dimension down: the x2 lines 1..n are split into layers by
the rule of Section 2 (boundary PML lines in the first and last layer), each
inner layer gets its own M, R and L problems with PML pads along x2, and one
application of Algorithm 2 over those inner layers stands in for H^-1.  The
cross axes of an inner problem are x1 (the boundary PML) and x3 (the outer
problem's own profile, auxiliary pads included).

To reuse the outer construction unchanged, the slab's unknowns are reordered
so that x2 is the slowest index: (i1, i3, i2), i1 fastest.  A slab line along
x2 is then a contiguous block of n * L unknowns, exactly as a grid line along
the sweep axis is for the whole problem.
"""
import numpy as np

from . import pml
from .operator import symmetric_operator
from .subproblem import Subproblem, _widths


class SlabProblem:
    """The slab of one 3D auxiliary problem, seen as a problem whose sweep
    axis is x2: it offers what the sweep construction reads from a Problem
    (sizes, partition settings, the operator on a range of x2 lines)."""

    def __init__(self, prob, sub, b2, gamma_aux2=None):
        self.outer = prob
        self.d = 3
        self.n = prob.n
        self.L3 = sub.L
        self.S = prob.n * sub.L               # unknowns on one x2 line: (i1, i3)
        self.N = self.S * prob.n
        self.b = b2
        self.gamma, self.C = prob.gamma, prob.C
        self.gamma_aux = prob.gamma if gamma_aux2 is None else int(gamma_aux2)
        self.h, self.omega = prob.h, prob.omega
        self.x1 = prob.cross                   # boundary PML along x1
        self.x3 = pml.tables(sub.lo, sub.hi, sub.phi, sub.psi, prob.C, _widths(prob, sub),
                             prob.h, prob.omega)
        # omega^2 / c^2 on the slab in (i1, i3, i2) order
        ksq = prob.ksq.reshape((prob.n, prob.n, prob.n), order="F")[:, :, sub.lo - 1:sub.hi]
        self.ksq = np.ascontiguousarray(ksq.transpose(0, 2, 1)).reshape(-1, order="F")

    def lines(self, vec, lo, hi):
        """Restriction of a reordered slab vector to x2 lines lo..hi."""
        return np.asarray(vec)[(lo - 1) * self.S: hi * self.S]

    def box_operator(self, lo, hi, phi, psi, widths=None):
        """Symmetric-form operator on x2 lines lo..hi of the slab (Dirichlet
        outside), the x2 profile vanishing on [phi, psi]."""
        x2 = pml.tables(lo, hi, phi, psi, self.C, widths or self.gamma, self.h, self.omega)
        return symmetric_operator([self.x1, self.x3, x2], self.lines(self.ksq, lo, hi), self.h)

    # slab order (i1, i2, i3) <-> sweep order (i1, i3, i2)
    def to_sweep(self, v):
        n, L = self.n, self.L3
        return np.asarray(v).reshape((L, n, n)).transpose(1, 0, 2).reshape(-1)

    def from_sweep(self, w):
        n, L = self.n, self.L3
        return np.asarray(w).reshape((n, L, n)).transpose(1, 0, 2).reshape(-1)


class RecursiveSubproblem(Subproblem):
    """A 3D auxiliary problem whose solve H^-1 g is replaced by one application
    of the additive sweeping preconditioner along x2 (inner layers of b2 lines,
    inner auxiliary PML of gamma_aux2 lines).  G~ (data placement and
    restriction) is the parent's."""

    def __init__(self, prob, sub, X_p, b2, gamma_aux2=None, factor=True):
        self.b2, self.gamma_aux2 = b2, gamma_aux2
        super().__init__(prob, sub, X_p, factor=factor)

    def factor(self):
        from .sweep import Preconditioner

        self.slab = SlabProblem(self.prob, self.sub, self.b2, self.gamma_aux2)
        self.inner = Preconditioner(self.slab)
        self.lu = self.inner                  # marks the problem as set up
        self.perm = None
        return self

    def solve(self, g):
        if self.lu is None:
            self.factor()
        s = self.slab
        return s.from_sweep(self.inner.apply(s.to_sweep(np.asarray(g, dtype=np.complex128))))
