"""Pins of oracle.pml against the printed PML profiles (Section 2: sigma, s;
Section 2.1: sigma^M_q, sigma^R_p, sigma^L_p)."""
import numpy as np
import pytest

from oracle import partition, pml

C, OMEGA = 25.0, 2 * np.pi * 8


def paper_sigma_global(x, eta):
    """Section 2 definition of sigma on [0, 1], written piecewise."""
    if x < eta:
        return (C / eta) * ((x - eta) / eta) ** 2
    if x <= 1 - eta:
        return 0.0
    return (C / eta) * ((x - 1 + eta) / eta) ** 2


@pytest.mark.parametrize("n,gamma", [(63, 12), (31, 8), (127, 9)])
def test_global_profile_matches_printed_formula(n, gamma):
    h = 1.0 / (n + 1)
    eta = gamma * h
    s_int, s_half = pml.global_axis(n, C, gamma, h, OMEGA)
    for i in range(1, n + 1):
        sig = paper_sigma_global(i * h, eta)
        assert s_int[i - 1] == pytest.approx(1 / (1 + 1j * sig / OMEGA), rel=1e-14)
    for k in range(n + 1):
        x = (k + 0.5) * h
        sig = paper_sigma_global(x, eta)
        assert s_half[k] == pytest.approx(1 / (1 + 1j * sig / OMEGA), rel=1e-14)


def test_closed_form_values():
    n, gamma = 63, 12
    h = 1.0 / (n + 1)
    eta = gamma * h
    # sigma = C/eta on the domain boundary (distance eta from the physical edge)
    assert pml.sigma(0.0, gamma, n + 1 - gamma, C, gamma, h) == pytest.approx(C / eta)
    assert pml.sigma(n + 1, gamma, n + 1 - gamma, C, gamma, h) == pytest.approx(C / eta)
    # zero on the physical region, including its edges
    t = np.linspace(gamma, n + 1 - gamma, 101)
    assert np.all(pml.sigma(t, gamma, n + 1 - gamma, C, gamma, h) == 0.0)
    # continuous and strictly increasing into the layer
    t = np.linspace(gamma - 1e-9, 0, 50)
    sig = pml.sigma(t, gamma, n + 1 - gamma, C, gamma, h)
    assert sig[0] < 1e-12 and np.all(np.diff(sig) > 0)
    # s = 1 where sigma = 0; |s| < 1 and Im s < 0 inside the layer
    s = pml.s(np.array([gamma + 0.5, 3.0]), gamma, n + 1 - gamma, C, gamma, h, OMEGA)
    assert s[0] == 1.0 and abs(s[1]) < 1 and s[1].imag < 0


def printed_aux_sigma(kind, p, t, gamma, b, m, eta):
    """Section 2.1 printed profiles (paper's partition, n = 2 gamma + m b - 2),
    written in grid units: x = t h, eta = gamma h, so every breakpoint is exact."""
    q = p
    one = 2 * gamma + m * b - 1          # x = 1 is line n + 1
    quad = lambda t0: (C / eta) * ((t - t0) / gamma) ** 2
    if kind == "M":
        if q == 1:
            if t < gamma:
                return quad(gamma)
            if t <= gamma + (b - 1):
                return 0.0
            return quad(gamma + (b - 1))
        if q == m:
            if t < one - gamma - (b - 1):
                return quad(one - gamma - (b - 1))
            if t <= one - gamma:
                return 0.0
            return quad(one - gamma)
        if t < gamma + (q - 1) * b:
            return quad(gamma + (q - 1) * b)
        if t <= gamma + (q * b - 1):
            return 0.0
        return quad(gamma + (q * b - 1))
    if kind == "R":
        if t < gamma + ((p - 1) * b - 1):
            raise AssertionError("outside D^R_p")
        if t <= gamma + (p * b - 1):
            return 0.0
        return quad(gamma + (p * b - 1))
    if kind == "L":
        if t > gamma + p * b:
            raise AssertionError("outside D^L_p")
        if t < gamma + (p - 1) * b:
            return quad(gamma + (p - 1) * b)
        return 0.0
    raise ValueError(kind)


@pytest.mark.parametrize("gamma,b,m", [(9, 8, 5), (12, 4, 6), (5, 3, 4)])
def test_auxiliary_profiles_match_printed_formulas(gamma, b, m):
    n = 2 * gamma + m * b - 2          # the paper's assumption in Section 2
    h = 1.0 / (n + 1)
    eta = gamma * h
    subs = partition.subproblems(n, b, gamma)
    assert len(subs["M"]) == m
    for kind in ("M", "R", "L"):
        for sub in subs[kind]:
            # integer and half lines of the extended grid, plus its Dirichlet lines
            ts = np.arange(2 * sub.lo - 2, 2 * sub.hi + 3) / 2.0
            for t in ts:
                want = printed_aux_sigma(kind, sub.p, t, gamma, b, m, eta)
                got = float(pml.sigma(t, sub.phi, sub.psi, C, gamma, h))
                assert got == pytest.approx(want, rel=1e-12, abs=1e-12), (kind, sub.p, t)


def test_two_sided_widths():
    """A profile with different widths below and above its zero region (a thin
    auxiliary pad on one side): each side is the quadratic of its own width,
    and equal widths give the one-width profile exactly."""
    from oracle import pml as P2
    h, C = 1.0 / 64, 25.0
    phi, psi = 10.0, 30.0
    t = np.array([4.0, 7.5, 10.0, 20.0, 30.0, 33.5, 36.0])
    sg = P2.sigma(t, phi, psi, C, (9, 5), h)
    e9, e5 = 9 * h, 5 * h
    ref = [(C / e9) * ((phi - x) * h / e9) ** 2 if x < phi else
           (C / e5) * ((x - psi) * h / e5) ** 2 if x > psi else 0.0 for x in t]
    np.testing.assert_allclose(sg, ref, rtol=1e-15, atol=0)
    np.testing.assert_array_equal(P2.sigma(t, phi, psi, C, (7, 7), h), P2.sigma(t, phi, psi, C, 7, h))
