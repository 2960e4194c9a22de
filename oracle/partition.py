"""Layer partition and extended grids along the sweep axis.  Parity pinned
(printed layer sizes of Sections 3.2 and 4.2, printed index sets of
Sections 2.1 and 3.1; tests/test_oracle_partition.py).

All indices are 1-based grid lines along the sweep axis (x2 in 2D, x3 in 3D,
Sections 3.1 and 4.1), inclusive ranges.  g = gamma - 1 is the number of grid
lines strictly inside one PML (sigma > 0): with eta = gamma*h the lines
1..gamma-1 carry sigma > 0 and line gamma is the first physical line.

Partition (Section 2, X_1..X_m; generalised to n != 2*gamma + m*b - 2 as the
experiments of Sections 3.2 and 4.2 require, where the first layer has b+gamma-1
lines and the last b+gamma-2):

    n_phys = n - 2g,  m = ceil(n_phys / b)
    X_1 = [1, g+b],  X_p = [gamma+(p-1)b, gamma+pb-1] (1<p<m),  X_m = [gamma+(m-1)b, n]

so the last layer holds r = n_phys - (m-1)b in [1, b] physical lines plus the
g PML lines; with n = 2*gamma + m*b - 2 this is exactly the paper's partition.

Arbitrary layer widths (Section 3.1 remarks: the subdomains need not have the
same width): b may instead be a list (w_1, ..., w_m) of physical lines per
layer, each >= 1, summing to n_phys.  With t_p = gamma + w_1 + ... + w_{p-1}
the first physical line of layer p,

    X_1 = [1, t_2 - 1],  X_p = [t_p, t_{p+1} - 1] (1<p<m),  X_m = [t_m, n];

the uniform rule is the list (b, ..., b, r).

Extended grids and the zero regions of their sweep-axis PML profiles
(Section 2.1 definitions of D^M_q, X^M_q, sigma^M_q, D^R_p, X^R_p, sigma^R_p,
D^L_p, X^L_p, sigma^L_p; the same sets in 2D and 3D):

    M_q: zero region [phi_q, psi_q],      lines [phi_q - g, psi_q + g]
    R_p: zero region [s_p - 1, psi_p],    lines [s_p, psi_p + g]        (p >= 2)
    L_p: zero region [phi_p, e_p + 1],    lines [phi_p - g, e_p]        (p <= m-1)

with [s_p, e_p] = X_p and its physical part phi_p = max(s_p, gamma),
psi_p = min(e_p, n+1-gamma).  sigma^R_p vanishes from the Dirichlet line
s_p - 1 (the left boundary of D^R_p) and sigma^L_p up to the Dirichlet line
e_p + 1 (the right boundary of D^L_p), as in their definitions.

Thinner auxiliary PML (Section 3.1 remarks, eta_aux < eta): a pad that faces a
neighbouring layer (not the boundary of the domain) has g_a = gamma_aux - 1
lines and the profile of width eta_aux = gamma_aux*h; a pad at the boundary of
the domain is the boundary PML itself (g lines, width eta).  With
gamma_aux = gamma every pad is as above.
"""
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Sub:
    kind: str   # "M", "R" or "L"
    p: int      # layer index, 1-based
    lo: int     # first grid line of the extended grid
    hi: int     # last grid line of the extended grid
    phi: float  # zero region of the sweep-axis PML profile
    psi: float
    gamma_lo: int = 0   # PML width (grid units) of the profile below phi / above psi
    gamma_hi: int = 0

    @property
    def L(self):
        return self.hi - self.lo + 1


def check_args(n, b, gamma):
    widths(n, b, gamma)


def widths(n, b, gamma):
    """Physical lines (w_1, ..., w_m) of the layers: the uniform rule for an
    integer b, else b itself after checking it."""
    if gamma < 2 or n - 2 * (gamma - 1) < 1:
        raise ValueError(f"invalid partition n={n} gamma={gamma}")
    n_phys = n - 2 * (gamma - 1)
    if isinstance(b, (int, np.integer)):
        if b < 1:
            raise ValueError(f"invalid layer width b={b}")
        m = -(-n_phys // b)
        return [int(b)] * (m - 1) + [n_phys - (m - 1) * int(b)]
    w = [int(x) for x in b]
    if not w or min(w) < 1 or sum(w) != n_phys:
        raise ValueError(f"layer widths {w} must be >= 1 and sum to n_phys = {n_phys}")
    return w


def layers(n, b, gamma):
    """[(s_p, e_p)] for p = 1..m."""
    w = widths(n, b, gamma)
    m = len(w)
    X, t = [], gamma
    for p in range(m):
        X.append((1 if p == 0 else t, n if p == m - 1 else t + w[p] - 1))
        t += w[p]
    return X


def physical(n, gamma, layer):
    s_p, e_p = layer
    return max(s_p, gamma), min(e_p, n + 1 - gamma)


def subproblems(n, b, gamma, gamma_aux=None):
    """Dict with lists 'M' (q=1..m), 'R' (p=2..m) and 'L' (p=1..m-1) of Sub."""
    X = layers(n, b, gamma)
    m = len(X)
    g = gamma - 1
    ga = gamma if gamma_aux is None else int(gamma_aux)
    if not 2 <= ga <= gamma:
        raise ValueError(f"invalid auxiliary PML width {gamma_aux} (gamma = {gamma})")
    # pad below layer p (toward layer p-1) and above it (toward layer p+1)
    low = lambda p: (g, gamma) if p == 1 else (ga - 1, ga)
    high = lambda p: (g, gamma) if p == m else (ga - 1, ga)
    M, R, L = [], [], []
    for q in range(1, m + 1):
        phi, psi = physical(n, gamma, X[q - 1])
        (gl, wl), (gh, wh) = low(q), high(q)
        M.append(Sub("M", q, phi - gl, psi + gh, phi, psi, wl, wh))
    for p in range(2, m + 1):
        s_p, _ = X[p - 1]
        _, psi = physical(n, gamma, X[p - 1])
        gh, wh = high(p)
        R.append(Sub("R", p, s_p, psi + gh, s_p - 1, psi, wh, wh))
    for p in range(1, m):
        _, e_p = X[p - 1]
        phi, _ = physical(n, gamma, X[p - 1])
        gl, wl = low(p)
        L.append(Sub("L", p, phi - gl, e_p, phi, e_p + 1, wl, wl))
    return {"M": M, "R": R, "L": L}
