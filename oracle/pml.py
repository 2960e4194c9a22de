"""PML profile.  Parity pinned (closed-form values, tests/test_oracle_pml.py).

Section 2 defines, for a PML of width eta = gamma*h,

    sigma(x) = (C/eta) * ((x - x_edge)/eta)^2   inside the layer,
    sigma(x) = 0                                 in the physical region,
    s(x)     = (1 + i sigma(x)/omega)^-1.

The auxiliary profiles sigma^M_q, sigma^R_p, sigma^L_p of Section 2.1 are the
same quadratic measured from the edge of their own zero region.  All of them
are therefore described here by the zero region [phi, psi], given in grid-line
units (x = t*h), and the grid coordinate t at which the profile is evaluated;
t may be a half-integer (eq. (1D): "the subscript i means evaluated at x = ih").
"""
import numpy as np


def sigma(t, phi, psi, C, gamma, h):
    """sigma at x = t*h for a profile that vanishes on [phi*h, psi*h].

    gamma is the PML width in grid units, or a pair (gamma below phi, gamma
    above psi) when the two sides differ (a thinner auxiliary PML facing the
    neighbouring layers, Section 3.1 remarks)."""
    t = np.asarray(t, dtype=np.float64)
    g_lo, g_hi = (gamma, gamma) if np.isscalar(gamma) else gamma
    if g_lo == g_hi:
        eta = g_lo * h
        dist = np.maximum(0.0, np.maximum(phi - t, t - psi)) * h   # distance to the zero region
        return (C / eta) * (dist / eta) ** 2
    eta_lo, eta_hi = g_lo * h, g_hi * h
    d_lo = np.maximum(0.0, phi - t) * h
    d_hi = np.maximum(0.0, t - psi) * h
    return (C / eta_lo) * (d_lo / eta_lo) ** 2 + (C / eta_hi) * (d_hi / eta_hi) ** 2


def s(t, phi, psi, C, gamma, h, omega):
    """s = (1 + i sigma/omega)^-1 at x = t*h."""
    return 1.0 / (1.0 + 1j * sigma(t, phi, psi, C, gamma, h) / omega)


def tables(lo, hi, phi, psi, C, gamma, h, omega):
    """s on the integer lines lo..hi and on the half lines lo-1/2 .. hi+1/2.

    Returns (s_int, s_half) with len(s_int) = hi-lo+1 and len(s_half) = hi-lo+2;
    s_half[k] is s at t = lo - 1/2 + k."""
    t_int = np.arange(lo, hi + 1, dtype=np.float64)
    t_half = np.arange(lo, hi + 2, dtype=np.float64) - 0.5
    return (s(t_int, phi, psi, C, gamma, h, omega),
            s(t_half, phi, psi, C, gamma, h, omega))


def global_axis(n, C, gamma, h, omega):
    """Tables of the boundary PML along one axis of the whole grid (lines 1..n).

    The physical region is [eta, 1-eta], i.e. lines gamma .. n+1-gamma."""
    return tables(1, n, gamma, n + 1 - gamma, C, gamma, h, omega)
