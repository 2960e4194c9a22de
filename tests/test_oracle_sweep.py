"""Pins of oracle.sweep (Algorithms 2 and 4):

* the accumulated O(m) sweeps equal the O(m^2) per-component recursion of
  Section 2.1 ("Accumulating the boundary values"), in 1D, 2D and 3D;
* one layer (m = 1) makes M^-1 = A^-1, so GMRES stops after one step;
* the preconditioner approximates G = A^-1 (the additive L + D + U splitting of
  eq. (LDUsplit)): on a point source in a smooth medium M^-1 f is close to
  A^-1 f, and a mistake in a sign, a boundary line or a sweep destroys that;
* at the paper's 2D settings (gamma = 9, b = 8, 8 points per wavelength,
  relative residual 1e-3, restart 40) GMRES needs no more iterations than the
  largest count printed in Tables 1-3.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads
from oracle import direct
from oracle.gmres import gmres
from oracle.operator import Problem
from oracle.sweep import Preconditioner

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("d,n,gamma,b", [(1, 60, 6, 4), (2, 31, 5, 3), (2, 40, 6, 5), (3, 13, 3, 2)])
def test_accumulated_sweep_equals_componentwise(d, n, gamma, b):
    rng = np.random.default_rng(n)
    c = 0.8 + 0.4 * rng.random((n,) * d)
    P = Problem(d, n, 2 * math.pi * (n + 1) / 10, gamma, 25.0, b, c)
    M = Preconditioner(P)
    assert M.m >= 3
    f = rng.standard_normal(P.N) + 1j * rng.standard_normal(P.N)
    z1, z2 = M.apply(f), M.apply_componentwise(f)
    assert np.linalg.norm(z1 - z2) <= 1e-12 * np.linalg.norm(z1)


@pytest.mark.parametrize("d,n,gamma,gamma_aux,b", [(2, 40, 6, 3, 5), (3, 15, 4, 2, 2)])
def test_accumulated_sweep_with_thin_auxiliary_pml(d, n, gamma, gamma_aux, b):
    """The accumulation identity holds for any auxiliary operators, so also
    with thinner auxiliary pads (Section 3.1 remarks)."""
    rng = np.random.default_rng(n + 1)
    c = 0.8 + 0.4 * rng.random((n,) * d)
    P = Problem(d, n, 2 * math.pi * (n + 1) / 10, gamma, 25.0, b, c, gamma_aux=gamma_aux)
    M = Preconditioner(P)
    assert M.m >= 3
    f = rng.standard_normal(P.N) + 1j * rng.standard_normal(P.N)
    z1, z2 = M.apply(f), M.apply_componentwise(f)
    assert np.linalg.norm(z1 - z2) <= 1e-12 * np.linalg.norm(z1)


@pytest.mark.parametrize("d,n,gamma,w", [(2, 40, 6, [3, 7, 1, 5, 6, 8]), (2, 31, 5, [2, 1, 6, 4, 10]),
                                         (3, 15, 3, [1, 4, 2, 4])])
def test_accumulated_sweep_with_arbitrary_widths(d, n, gamma, w):
    """Layers of unequal widths (Section 3.1 remarks): the accumulation
    identity does not depend on the widths."""
    rng = np.random.default_rng(n + 7)
    c = 0.8 + 0.4 * rng.random((n,) * d)
    P = Problem(d, n, 2 * math.pi * (n + 1) / 10, gamma, 25.0, w, c)
    M = Preconditioner(P)
    assert M.m == len(w)
    f = rng.standard_normal(P.N) + 1j * rng.standard_normal(P.N)
    z1, z2 = M.apply(f), M.apply_componentwise(f)
    assert np.linalg.norm(z1 - z2) <= 1e-12 * np.linalg.norm(z1)


def test_one_layer_of_full_width_is_exact():
    n, gamma = 24, 5
    P = Problem(2, n, 2 * math.pi * 2, gamma, 25.0, [n - 2 * (gamma - 1)],
                1.0 + 0.1 * np.random.default_rng(3).random((n, n)))
    M = Preconditioner(P)
    assert M.m == 1
    b = np.random.default_rng(4).standard_normal(P.N) + 0j
    np.testing.assert_allclose(M.apply(b), direct.solve(P.A(), b), rtol=1e-10, atol=1e-14)


def test_unequal_widths_keep_the_iteration_band():
    """Wider layers across the lens and thinner ones elsewhere (widths 4..16
    at gamma = 9, n = 127): GMRES(40) to 1e-3 stays within the largest count
    printed in Tables 1-3."""
    table = json.load(open(os.path.join(GOLDEN, "paper_iterations.json")))
    largest = max(max(v) for fam in ("lens", "waveguide", "random") for v in table[fam].values())
    w = workloads.paper_workload("lens", 127)
    w["b"] = [4, 8, 16, 12, 16, 16, 8, 8, 4, 4, 6, 9]
    assert sum(w["b"]) == 127 - 16
    P = Problem.from_workload(w)
    A = P.A()
    M = Preconditioner(P)
    for k in range(2):
        b = w["f"][k] / P.scale()
        x, it, rr, _ = gmres(lambda v: A @ v, M.apply, b, w["tol"], w["restart"], 100)
        assert rr <= w["tol"] and 1 <= it <= largest


def test_thin_auxiliary_pml_keeps_the_iteration_band():
    """eta_aux = 5h with eta = 9h (the paper's 3D choice) at the 2D paper
    settings, n = 127: still within the largest printed count."""
    table = json.load(open(os.path.join(GOLDEN, "paper_iterations.json")))
    largest = max(max(v) for fam in ("lens", "waveguide", "random") for v in table[fam].values())
    w = workloads.paper_workload("lens", 127)
    w["gamma_aux"] = 5
    P = Problem.from_workload(w)
    A = P.A()
    M = Preconditioner(P)
    for k in range(2):
        b = w["f"][k] / P.scale()
        x, it, rr, _ = gmres(lambda v: A @ v, M.apply, b, w["tol"], w["restart"], 100)
        assert rr <= w["tol"] and 1 <= it <= largest


@pytest.mark.parametrize("field", list(workloads.PAPER_FIELDS))
def test_paper_3d_workloads_within_printed_band(field):
    """The 3D paper-settings problems (eta = 9h, eta_aux = 5h, b = 4) of every
    field and both forces at n = 23 stay within the largest count printed in
    Tables 4-6."""
    table = json.load(open(os.path.join(GOLDEN, "paper_iterations_3d.json")))
    largest = max(max(v) for fam in ("lens", "waveguide", "random") for v in table[fam].values())
    w = workloads.paper_workload3d(field, 23)
    P = Problem.from_workload(w)
    A = P.A()
    M = Preconditioner(P)
    for k in range(2):
        b = w["f"][k] / P.scale()
        x, it, rr, _ = gmres(lambda v: A @ v, M.apply, b, w["tol"], w["restart"], 100)
        assert rr <= w["tol"]
        assert 1 <= it <= largest, (field, k, it)


def test_single_layer_is_exact():
    n, gamma = 20, 6
    P = Problem(2, n, 2 * math.pi * 2, gamma, 25.0, 20, 1.0 + 0.1 * np.random.default_rng(1).random((n, n)))
    M = Preconditioner(P)
    assert M.m == 1
    A = P.A()
    b = np.random.default_rng(2).standard_normal(P.N) + 0j
    np.testing.assert_allclose(M.apply(b), direct.solve(A, b), rtol=1e-10, atol=1e-14)
    x, it, rr, _ = gmres(lambda v: A @ v, M.apply, b, 1e-10, 20, 20)
    assert it == 1 and rr <= 1e-10


def _point_source_case(n, freq, gamma, b, velocity):
    omega = 2 * math.pi * freq
    c = workloads.velocity_lens2d(n) if velocity == "lens" else workloads.velocity_constant(n, 2)
    P = Problem(2, n, omega, gamma, 25.0, b, c)
    f = workloads.flat(workloads.gaussian_source(n, 2, omega, (0.5, 0.125)))
    return P, f / P.scale()


@pytest.mark.parametrize("velocity,bound", [("constant", 3e-2), ("lens", 3e-2)])
def test_preconditioner_approximates_green(velocity, bound):
    P, b = _point_source_case(127, 16, 9, 8, velocity)
    M = Preconditioner(P)
    u = direct.solve(P.A(), b)
    err = np.linalg.norm(M.apply(b) - u) / np.linalg.norm(u)
    assert err < bound


def test_iterations_within_printed_band():
    table = json.load(open(os.path.join(GOLDEN, "paper_iterations.json")))
    largest = max(max(v) for fam in ("lens", "waveguide", "random") for v in table[fam].values())
    for n, freq in zip(table["n"][:2], table["omega_over_2pi"][:2]):
        P, b = _point_source_case(n, freq, 9, 8, "lens")
        A = P.A()
        M = Preconditioner(P)
        x, it, rr, _ = gmres(lambda v: A @ v, M.apply, b, 1e-3, 40, 100)
        assert rr <= 1e-3
        assert 1 <= it <= largest, (n, it)


@pytest.mark.parametrize("field", list(workloads.PAPER_FIELDS))
def test_paper_workloads_within_printed_band(field):
    """The paper-settings problems of every field (lens, waveguide, random) and
    both forces (point source, wave packet) at n = 127 stay within the largest
    count printed in Tables 1-3."""
    table = json.load(open(os.path.join(GOLDEN, "paper_iterations.json")))
    largest = max(max(v) for fam in ("lens", "waveguide", "random") for v in table[fam].values())
    w = workloads.paper_workload(field, 127)
    P = Problem.from_workload(w)
    A = P.A()
    M = Preconditioner(P)
    for k in range(2):
        b = w["f"][k] / P.scale()
        x, it, rr, _ = gmres(lambda v: A @ v, M.apply, b, w["tol"], w["restart"], 100)
        assert rr <= w["tol"]
        assert 1 <= it <= largest, (field, k, it)


def test_one_dimension_is_nearly_exact():
    """In 1D the auxiliary PMLs absorb the transmitted wave almost perfectly, so
    the additive splitting is close to exact."""
    n = 255
    P = Problem(1, n, 2 * math.pi * 32, 9, 25.0, 8, np.ones(n))
    rng = np.random.default_rng(4)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    M = Preconditioner(P)
    u = direct.solve(P.A(), b)
    assert np.linalg.norm(M.apply(b) - u) / np.linalg.norm(u) < 1e-2
