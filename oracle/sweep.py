"""The additive sweeping preconditioner: setup (Algorithms 1 and 3) and apply
(Algorithms 2 and 4).  Parity pinned (the O(m^2) per-component recursion of
Section 2.1 it must equal exactly; m = 1 gives A^-1; the iteration counts of
Tables 1-3 at the paper's settings; tests/test_oracle_sweep.py).

Notation follows Section 2.1 ("Accumulating the boundary values") and the
"Putting together" paragraph of Section 3.1: for a vector on X_p (column-major,
sweep axis slowest) its left boundary value g^L is the first grid line and its
right boundary value g^R the last one.
"""
import numpy as np

from . import partition
from .subproblem import Subproblem


class Preconditioner:
    """M^-1 for the symmetric-form system of ``prob`` (an operator.Problem).

    keep_factors=False factors each subproblem when it is used and drops it
    afterwards: same arithmetic, bounded memory, for large grids.

    inner=(b2, gamma_aux2), 3D only: every auxiliary problem is solved by the
    additive sweeping preconditioner along x2 (inner layers of b2 lines, inner
    auxiliary PML of gamma_aux2 lines) instead of exactly (Section 5;
    recursive.RecursiveSubproblem)."""

    def __init__(self, prob, keep_factors=True, inner=None):
        self.prob = prob
        self.X = partition.layers(prob.n, prob.b, prob.gamma)
        self.m = len(self.X)
        subs = partition.subproblems(prob.n, prob.b, prob.gamma, prob.gamma_aux)
        self.keep = keep_factors
        # Algorithm 1 / 3: factor H^M_q (q=1..m), H^R_p (p=2..m), H^L_p (p=1..m-1).
        if inner is None:
            mk = lambda s: Subproblem(prob, s, self.X[s.p - 1], factor=keep_factors)
        else:
            from .recursive import RecursiveSubproblem

            if prob.d != 3:
                raise ValueError("the recursive sweep applies to 3D problems")
            mk = lambda s: RecursiveSubproblem(prob, s, self.X[s.p - 1], *inner, factor=keep_factors)
        self.M = {s.p: mk(s) for s in subs["M"]}
        self.R = {s.p: mk(s) for s in subs["R"]}
        self.L = {s.p: mk(s) for s in subs["L"]}

    # -- pieces -------------------------------------------------------------------------
    def layer(self, vec, p):
        s_p, e_p = self.X[p - 1]
        return self.prob.lines(vec, s_p, e_p)

    def left(self, v):
        return v[: self.prob.S]

    def right(self, v):
        return v[-self.prob.S:]

    def _G(self, sp_, data):
        out = sp_.G(data)
        if not self.keep:
            sp_.lu = None
        return out

    def GM(self, q, y):
        return self._G(self.M[q], y)

    def GR(self, p, w):
        return self._G(self.R[p], w)

    def GL(self, p, w):
        return self._G(self.L[p], w)

    # -- Algorithm 2 / 4 -------------------------------------------------------------------
    def _sweep(self, u_qq, order, G, exit_line):
        """One directional sweep of Section 2.1 ("Accumulating the boundary
        values"): walking the layers in `order`, the first layer hands on the
        exit line of its own local solution; every later layer p solves its
        auxiliary problem with the accumulated line as boundary data (the part
        of u~_p due to the sources behind it) and hands on the exit line of that
        part plus that of u~_{p,p}.  Returns {p: part of u~_p from behind}."""
        part = {}
        line = exit_line(u_qq[order[0]])
        for p in order[1:]:
            part[p] = G(p, line)
            line = exit_line(part[p]) + exit_line(u_qq[p])
        return part

    def apply(self, f):
        """u~ = M^-1 f (Algorithms 2 and 4): the local solves u~_{p,p} = G~^M_p f_p,
        the two sweeps, and u~_p as the sum of the local part and the parts
        arriving from either side (one of them at the first and last layer)."""
        m = self.m
        f = np.asarray(f, dtype=np.complex128)
        u_qq = {q: self.GM(q, self.layer(f, q)) for q in range(1, m + 1)}
        # right-going: data enters R_p on its first line, leaves on the last
        from_left = self._sweep(u_qq, list(range(1, m + 1)), self.GR, self.right)
        # left-going: data enters L_p on its last line, leaves on the first
        from_right = self._sweep(u_qq, list(range(m, 0, -1)), self.GL, self.left)
        out = []
        for p in range(1, m + 1):
            v = u_qq[p].copy()
            if p > 1:
                v = from_left[p] + v
            if p < m:
                v = v + from_right[p]
            out.append(v)
        return np.concatenate(out)

    def apply_componentwise(self, f):
        """The O(m^2) form of Section 2.1: every u~_{p,q} by its own recursion,
        u~_{p,q} = G~^R_p u~^R_{p-1,q} (p > q), G~^L_p u~^L_{p+1,q} (p < q),
        then u~_p = sum_q u~_{p,q}."""
        m = self.m
        f = np.asarray(f, dtype=np.complex128)
        total = {p: 0 for p in range(1, m + 1)}
        for q in range(1, m + 1):
            u = {q: self.GM(q, self.layer(f, q))}
            for p in range(q + 1, m + 1):
                u[p] = self.GR(p, self.right(u[p - 1]))
            for p in range(q - 1, 0, -1):
                u[p] = self.GL(p, self.left(u[p + 1]))
            for p in range(1, m + 1):
                total[p] = total[p] + u[p]
        return np.concatenate([total[p] for p in range(1, m + 1)])
