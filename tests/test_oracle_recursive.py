"""Pins of the recursive sweep of the 3D auxiliary problems (Section 5: the
quasi-2D problems solved by sweeping along x2 with the same technique).

* one inner layer: the inner preconditioner's only problem is the slab problem
  itself, so the recursive G~ equals the exact G~ (any mistake in the slab
  reordering, its tables or its data placement breaks this);
* the reordered slab operator over every x2 line equals the auxiliary
  problem's H with rows and columns permuted;
* the inner apply (Algorithm 2 along x2) equals its O(m^2) per-component form;
* with several inner layers the recursive G~ approximates the exact one
  (measured 0.3-2.1% on random data at n = 15);
* at the 3D experiments' settings (eta 9h, eta_aux 5h, b 4) outer GMRES with
  recursive inner solves stays within the largest count of Tables 4-6 and
  within one iteration of the exact preconditioner's count."""
import json
import math
import os

import numpy as np
import pytest

import workloads
from oracle import partition
from oracle.gmres import gmres
from oracle.operator import Problem
from oracle.recursive import RecursiveSubproblem, SlabProblem
from oracle.subproblem import Subproblem
from oracle.sweep import Preconditioner

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _problem(n=15, gamma=4, b=4):
    c = workloads.velocity_lens3d(n)
    return Problem(3, n, 2 * math.pi * (n + 1) / 8, gamma, 25.0, b, c)


def _data(P, X, s, rng):
    k = P.S * (X[s.p - 1][1] - X[s.p - 1][0] + 1) if s.kind == "M" else P.S
    return rng.standard_normal(k) + 1j * rng.standard_normal(k)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("kind", ["M", "R", "L"])
def test_one_inner_layer_is_exact(kind):
    P = _problem()
    X = partition.layers(P.n, P.b, P.gamma)
    subs = partition.subproblems(P.n, P.b, P.gamma)
    rng = np.random.default_rng(1)
    n_phys = P.n - 2 * (P.gamma - 1)
    for s in (subs[kind][0], subs[kind][-1]):
        rc = RecursiveSubproblem(P, s, X[s.p - 1], n_phys)
        assert rc.inner.m == 1
        d = _data(P, X, s, rng)
        assert rel(rc.G(d), Subproblem(P, s, X[s.p - 1]).G(d)) < 1e-12, (kind, s.p)


def test_slab_reordering_reproduces_H():
    P = _problem()
    X = partition.layers(P.n, P.b, P.gamma)
    rng = np.random.default_rng(2)
    for s in partition.subproblems(P.n, P.b, P.gamma)["M"][:2]:
        slab = SlabProblem(P, s, 4)
        H = Subproblem(P, s, X[s.p - 1], factor=False).H
        Hs = slab.box_operator(1, P.n, P.gamma, P.n + 1 - P.gamma)
        v = rng.standard_normal(H.shape[0]) + 1j * rng.standard_normal(H.shape[0])
        assert np.array_equal(slab.from_sweep(slab.to_sweep(v)), v)
        assert rel(Hs @ slab.to_sweep(v), slab.to_sweep(H @ v)) < 1e-14
        # x1 stays the fastest index: a slab line along x1 stays contiguous
        e = np.zeros(H.shape[0])
        e[: P.n] = 1.0
        assert np.array_equal(slab.to_sweep(e)[: P.n], np.ones(P.n))


def test_inner_apply_equals_componentwise():
    P = _problem()
    s = partition.subproblems(P.n, P.b, P.gamma)["M"][1]
    slab = SlabProblem(P, s, 2)
    M = Preconditioner(slab)
    assert M.m >= 3
    rng = np.random.default_rng(3)
    g = rng.standard_normal(slab.N) + 1j * rng.standard_normal(slab.N)
    assert rel(M.apply(g), M.apply_componentwise(g)) < 1e-12


@pytest.mark.parametrize("b2", [2, 4])
def test_recursive_approximates_exact_green(b2):
    P = _problem()
    X = partition.layers(P.n, P.b, P.gamma)
    subs = partition.subproblems(P.n, P.b, P.gamma)
    rng = np.random.default_rng(4)
    for kind in ("M", "R", "L"):
        s = subs[kind][0]
        rc = RecursiveSubproblem(P, s, X[s.p - 1], b2)
        assert rc.inner.m > 1
        d = _data(P, X, s, rng)
        e = rel(rc.G(d), Subproblem(P, s, X[s.p - 1]).G(d))
        assert 1e-6 < e < 5e-2, (kind, e)      # an approximation, and a close one


@pytest.mark.parametrize("field", list(workloads.PAPER_FIELDS))
def test_recursive_paper_3d_within_printed_band(field):
    table = json.load(open(os.path.join(GOLDEN, "paper_iterations_3d.json")))
    largest = max(max(v) for fam in ("lens", "waveguide", "random") for v in table[fam].values())
    w = workloads.paper_workload3d(field, 23)
    P = Problem.from_workload(w)
    A = P.A()
    exact = Preconditioner(P)
    rec = Preconditioner(P, inner=(w["b"], w["gamma_aux"]))
    for k in range(2):
        b = w["f"][k] / P.scale()
        _, it_x, _, _ = gmres(lambda v: A @ v, exact.apply, b, w["tol"], w["restart"], 100)
        _, it_r, rr, _ = gmres(lambda v: A @ v, rec.apply, b, w["tol"], w["restart"], 100)
        assert rr <= w["tol"]
        assert 1 <= it_r <= largest and it_x <= it_r <= it_x + 1, (field, k, it_x, it_r)


def test_recursive_needs_3d():
    w = workloads.workload("2d_n63_const", n=31)
    with pytest.raises(ValueError):
        Preconditioner(Problem.from_workload(w), inner=(4, 12))
