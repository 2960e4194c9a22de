"""The discrete PML-Helmholtz operator.  Parity pinned (sine-mode eigenvalues
with the PML switched off, exact symmetry, and the pointwise unsymmetrized
equation of the paper; tests/test_oracle_operator.py).

Eq. (1D) of Section 2, eq. (2D) of Section 3.1 and eq. (3D) of Section 4.1
are the centered scheme

    sum_k  s_k(i)/h * ( s_k(i+1/2)/h (u_{i+e_k} - u_i) - s_k(i-1/2)/h (u_i - u_{i-e_k}) )
      + omega^2 / c_i^2 u_i = f_i ,

with u = 0 outside the grid; the experiments put a PML on every side
(Sections 3.2 and 4.2), so every axis k carries its own s_k.  The symmetric
version mentioned in Section 3.1 (remark 4) divides row i by prod_k s_k(i_k):

    A_sym = sum_k ( x_{j != k} diag(1/s_j) ) (x) T_k  +  diag(omega^2 / (c^2 prod_k s_k)),
    (T_k u)_i = ( s_k(i+1/2)(u_{i+1} - u_i) - s_k(i-1/2)(u_i - u_{i-1}) ) / h^2 ,

which is complex symmetric (A_sym = A_sym^T) and has the same solution u for
the right-hand side f / prod_k s_k.  Unknowns are ordered column-major
(first index fastest), as in Sections 3.1 and 4.1.
"""
import numpy as np
import scipy.sparse as sp

from . import pml


def second_difference(s_half, h):
    """T for one axis: s_half[k] is s at the half line between unknowns k-1 and k
    (0-based), so len(s_half) = (number of unknowns) + 1."""
    s_half = np.asarray(s_half, dtype=np.complex128)
    main = -(s_half[:-1] + s_half[1:]) / h ** 2
    off = s_half[1:-1] / h ** 2
    return sp.diags([off, main, off], [-1, 0, 1], format="csr")


def _kron_cols(mats):
    """Kronecker product with the first factor acting on the fastest index."""
    out = mats[-1]
    for a in reversed(mats[:-1]):
        out = sp.kron(out, a, format="csr")
    return out


def _kron_vec(vecs):
    out = np.asarray(vecs[-1])
    for v in reversed(vecs[:-1]):
        out = np.kron(out, v)
    return out


def symmetric_operator(axes, ksq, h):
    """A_sym on a box grid.

    axes -- per axis (fastest first) a pair (s_int, s_half) of s on the
            unknowns' lines and on the half lines around them;
    ksq  -- omega^2/c^2 on the box, column-major."""
    d = len(axes)
    A = None
    for k in range(d):
        mats = []
        for j in range(d):
            s_int, s_half = axes[j]
            mats.append(second_difference(s_half, h) if j == k
                        else sp.diags(1.0 / np.asarray(s_int)))
        term = _kron_cols(mats)
        A = term if A is None else A + term
    prod_s = _kron_vec([np.asarray(a[0]) for a in axes])
    return (A + sp.diags(np.asarray(ksq) / prod_s)).tocsr()


class Problem:
    """The discretized problem of Section 1 with PML on all sides.

    d, n, omega as in the paper; gamma is the PML width in grid units
    (eta = gamma*h); C the PML constant; b the lines per interior layer, or a
    list of physical lines per layer (arbitrary widths, Section 3.1 remarks);
    c the velocity on the (n,)*d grid (first index = x1); gamma_aux the width of
    the auxiliary PML pads facing neighbouring layers (None: gamma)."""

    def __init__(self, d, n, omega, gamma, C, b, c, pml_axes="all", gamma_aux=None):
        self.d, self.n, self.omega = int(d), int(n), float(omega)
        self.gamma, self.C = int(gamma), float(C)
        self.b = int(b) if isinstance(b, (int, np.integer)) else tuple(int(x) for x in b)
        self.gamma_aux = self.gamma if gamma_aux is None else int(gamma_aux)
        self.h = 1.0 / (self.n + 1)
        c = np.asarray(c, dtype=np.float64).reshape((self.n,) * self.d)
        self.c = c
        self.ksq = (self.omega ** 2 / c ** 2).reshape(-1, order="F")
        self.axis = pml.global_axis(self.n, self.C, self.gamma, self.h, self.omega)
        # The experiments put the PML on every side (Sections 3.2, 4.2); the
        # derivations of Sections 3.1 and 4.1 put it on the two sweep-end sides
        # only, which pml_axes="sweep" reproduces (cross axes get s = 1).
        if pml_axes == "all":
            self.cross = self.axis
        elif pml_axes == "sweep":
            self.cross = (np.ones(self.n, np.complex128), np.ones(self.n + 1, np.complex128))
        else:
            raise ValueError(pml_axes)
        self.N = self.n ** self.d
        self.S = self.n ** (self.d - 1)   # unknowns on one line (cross-section)

    @classmethod
    def from_workload(cls, w):
        return cls(w["d"], w["n"], w["omega"], w["gamma"], w["C"], w["b"], w["c"],
                   gamma_aux=w.get("gamma_aux"))

    def axes(self):
        """Per-axis (s_int, s_half), fastest axis first; the sweep axis is last."""
        return [self.cross] * (self.d - 1) + [self.axis]

    def A(self):
        """Global symmetric-form operator."""
        return symmetric_operator(self.axes(), self.ksq, self.h)

    def scale(self):
        """prod_k s_k(i_k) on the grid: the symmetric right-hand side is f / scale()."""
        return _kron_vec([a[0] for a in self.axes()])

    def lines(self, vec, lo, hi):
        """Restriction of a grid vector to sweep lines lo..hi (1-based, inclusive)."""
        return np.asarray(vec)[(lo - 1) * self.S: hi * self.S]

    def box_operator(self, lo, hi, phi, psi, widths=None):
        """Symmetric-form operator on sweep lines lo..hi with Dirichlet data
        outside, the boundary PML on the cross axes and, on the sweep axis, the
        profile that vanishes on [phi, psi] (widths: its PML width below phi and
        above psi, default gamma on both sides)."""
        sweep = pml.tables(lo, hi, phi, psi, self.C, widths or self.gamma, self.h, self.omega)
        ksq = self.lines(self.ksq, lo, hi)
        return symmetric_operator([self.cross] * (self.d - 1) + [sweep], ksq, self.h)
