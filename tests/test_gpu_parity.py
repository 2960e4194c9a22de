"""GPU parity of the HIP path (through the C ABI) against the CPU FP64 oracle.

Tolerances (relative 2-norm unless stated):
* stencil y = A x, complex double: 1e-13;
* one auxiliary Green's operator and the whole apply, FP64 factors: 1e-11;
  FP32 factors: 7e-6 per operator and 8e-6 for the apply (about ten times the
  largest errors measured on these cases, 6.7e-7 and 7.5e-7);
* GMRES to tol 1e-6: iteration count within +-1 of the oracle's; the solution
  within 1e-6 of the oracle's (FP64) and within 1e-5 (FP32 factors: two valid
  solutions at tol 1e-6 may differ by up to cond(A) 1e-6; the 1e-6 solution
  gate at tol 1e-10 is in test_gpu_headline.py); the true relative residual,
  recomputed by the oracle's operator, <= 1e-6.
The grids span many layers, thin and thick auxiliary problems (L = 12..26), and
a ragged last layer (n = 100: r = 2 physical lines in X_m)."""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import direct, partition
from oracle.gmres import gmres as oracle_gmres
from oracle.operator import Problem
from oracle.subproblem import Subproblem
from oracle.sweep import Preconditioner

pytestmark = pytest.mark.gpu
asp = pytest.importorskip("paper_1504_04058_amd.asp")

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _problem(n, gamma, b, velocity="random", freq=None, seed=1):
    d = 2
    omega = 2 * math.pi * (freq if freq is not None else (n + 1) / 8)
    if velocity == "random":
        c = workloads.velocity_random(n, d, seed=seed)
    elif velocity == "lens":
        c = workloads.velocity_lens2d(n)
    else:
        c = workloads.velocity_constant(n, d)
    return Problem(d, n, omega, gamma, 25.0, b, c)


def _plan(P, prec=asp.ASP_PREC_FP64):
    return asp.Plan(P.d, P.c, P.omega, P.n, P.b, P.gamma, C=P.C, prec=prec)


CASES = [(63, 12, 4), (100, 12, 4), (127, 9, 8), (48, 5, 3)]


@pytest.mark.parametrize("n,gamma,b", CASES)
def test_stencil(n, gamma, b):
    P = _problem(n, gamma, b)
    rng = np.random.default_rng(n)
    x = rng.standard_normal((3, P.N)) + 1j * rng.standard_normal((3, P.N))
    with _plan(P) as plan:
        y = host(plan.matvec(dev(x)))
    A = P.A()
    for r in range(3):
        assert rel(y[r], A @ x[r]) < 1e-13


@pytest.mark.parametrize("n,gamma", [(15, 3), (31, 8)])
def test_stencil_3d(n, gamma):
    rng = np.random.default_rng(n)
    c = 1.0 + 0.3 * rng.random((n, n, n))
    P = Problem(3, n, 2 * math.pi * 3, gamma, 25.0, 4, c)
    x = rng.standard_normal((2, P.N)) + 1j * rng.standard_normal((2, P.N))
    with asp.Plan(3, c, P.omega, n, 4, gamma) as plan:
        y = host(plan.matvec(dev(x)))
    A = P.A()
    for r in range(2):
        assert rel(y[r], A @ x[r]) < 1e-13


# BF16X3 (real-split bf16 products, FP32 factors and accumulation): measured
# at most 1.6e-5 for the operators and 1.8e-5 for the apply over these cases
@pytest.mark.parametrize("prec,tol", [(asp.ASP_PREC_FP64, 1e-11), (asp.ASP_PREC_FP32, 7e-6),
                                      (asp.ASP_PREC_BF16X3, 1e-4)])
@pytest.mark.parametrize("n,gamma,b", CASES)
def test_auxiliary_operators(n, gamma, b, prec, tol):
    P = _problem(n, gamma, b)
    X = partition.layers(n, b, gamma)
    subs = partition.subproblems(n, b, gamma)
    m = len(X)
    rng = np.random.default_rng(7)
    picks = {"M": [1, 2, m // 2, m], "R": [2, m // 2, m], "L": [1, m // 2, m - 1]}
    kinds = {"M": asp.ASP_SUB_M, "R": asp.ASP_SUB_R, "L": asp.ASP_SUB_L}
    with _plan(P, prec) as plan:
        plan.factor()
        for kind, ps in picks.items():
            for p in sorted(set(ps)):
                sub = [s for s in subs[kind] if s.p == p][0]
                ref = Subproblem(P, sub, X[p - 1])
                Np = P.S * (X[p - 1][1] - X[p - 1][0] + 1)
                k_in = Np if kind == "M" else P.S
                data = rng.standard_normal((2, k_in)) + 1j * rng.standard_normal((2, k_in))
                out = host(plan.subsolve(kinds[kind], p, dev(data), Np)).reshape(2, Np)
                for r in range(2):
                    e = rel(out[r], ref.G(data[r]))
                    print(f"2D G~{kind}_{p} n={n} prec={prec}: rel err {e:.2e}", flush=True)
                    assert e < tol, (kind, p)


@pytest.mark.parametrize("prec,tol", [(asp.ASP_PREC_FP64, 1e-11), (asp.ASP_PREC_FP32, 8e-6),
                                      (asp.ASP_PREC_BF16X3, 1e-4)])
@pytest.mark.parametrize("n,gamma,b", CASES)
def test_apply(n, gamma, b, prec, tol):
    P = _problem(n, gamma, b)
    M = Preconditioner(P)
    rng = np.random.default_rng(3)
    r = rng.standard_normal((2, P.N)) + 1j * rng.standard_normal((2, P.N))
    with _plan(P, prec) as plan:
        plan.factor()
        z = host(plan.apply(dev(r)))
    for k in range(2):
        e = rel(z[k], M.apply(r[k]))
        print(f"2D apply n={n} gamma={gamma} b={b} prec={prec}: rel err {e:.2e}", flush=True)
        assert e < tol


@pytest.mark.parametrize("prec,tol", [(asp.ASP_PREC_FP64, 1e-11), (asp.ASP_PREC_FP32, 1e-5)])
def test_apply_odd_batch_count_per_sweep_wavefront(prec, tol):
    """n = 300: each of the eight wavefronts of a sweep step takes 48 columns
    of the boundary map, three batches of 16, so the second register slot's
    last batch lies wholly past the wavefront's range and must add nothing;
    the seventh wavefront's range ends past n and the eighth lies wholly past
    it."""
    n, gamma, b = 300, 12, 4
    assert (n + 127) // 128 * 16 == 48 and 6 * 48 < n < 7 * 48
    P = _problem(n, gamma, b)
    M = Preconditioner(P)
    rng = np.random.default_rng(5)
    r = rng.standard_normal((2, P.N)) + 1j * rng.standard_normal((2, P.N))
    with _plan(P, prec) as plan:
        plan.factor()
        z = host(plan.apply(dev(r)))
    for k in range(2):
        e = rel(z[k], M.apply(r[k]))
        print(f"2D apply n=300 prec={prec}: rel err {e:.2e}", flush=True)
        assert e < tol


def test_single_and_two_layers():
    for n, gamma, b in [(16, 5, 8), (17, 5, 8)]:     # m = 1 and m = 2
        P = _problem(n, gamma, b, velocity="constant", freq=2)
        M = Preconditioner(P)
        assert M.m == (1 if n == 16 else 2)
        r = np.random.default_rng(0).standard_normal(P.N) + 0j
        with _plan(P) as plan:
            plan.factor()
            z = host(plan.apply(dev(r[None])))[0]
        assert rel(z, M.apply(r)) < 1e-11
        if M.m == 1:
            assert rel(z, direct.solve(P.A(), r)) < 1e-10


@pytest.mark.parametrize("prec,tol", [(asp.ASP_PREC_FP64, 1e-11), (asp.ASP_PREC_FP32, 8e-6)])
def test_three_and_four_layers(prec, tol):
    """m = 3 and 4: one and two boundary-map problems per sweep (the
    smallest launches of the diagonal-block recurrence and of the map
    solves), against the oracle."""
    for n, gamma, b, m in [(25, 5, 8, 3), (33, 5, 8, 4)]:
        P = _problem(n, gamma, b)
        M = Preconditioner(P)
        assert M.m == m
        r = np.random.default_rng(1).standard_normal((3, P.N)) + 1j * np.random.default_rng(2).standard_normal((3, P.N))
        with _plan(P, prec) as plan:
            plan.factor()
            z = host(plan.apply(dev(r)))
        for k in range(3):
            e = rel(z[k], M.apply(r[k]))
            print(f"2D apply m={m} n={n} prec={prec}: rel err {e:.2e}", flush=True)
            assert e < tol


def _oracle_solve(P, b, tol, restart):
    A = P.A()
    M = Preconditioner(P)
    x, it, rr, hist = oracle_gmres(lambda v: A @ v, M.apply, b, tol, restart, 200, record=True)
    return A, x, it, rr, hist


@pytest.mark.parametrize("prec,soltol", [(asp.ASP_PREC_FP64, 1e-6), (asp.ASP_PREC_FP32, 1e-5)])
def test_gmres_small_config(prec, soltol):
    """2D n = 63, constant c, omega = 2 pi 8, gamma = 12, b = 4, GMRES(20), tol 1e-6."""
    w = workloads.workload("2d_n63_const")
    P = Problem.from_workload(w)
    b = w["f"][0] / P.scale()
    A, x_ref, it_ref, rr_ref, hist = _oracle_solve(P, b, w["tol"], w["restart"])
    with _plan(P, prec) as plan:
        u, it, rr, st = plan.gmres(dev(w["f"]), tol=w["tol"], restart=w["restart"], maxit=200)
        u = host(u)[0]
    assert st == asp.ASP_OK
    assert abs(int(it[0]) - it_ref) <= 1
    assert np.linalg.norm(b - A @ u) / np.linalg.norm(b) <= w["tol"] * (1 + 1e-9)
    assert rel(u, x_ref) < soltol


@pytest.mark.parametrize("prec", [asp.ASP_PREC_FP64, asp.ASP_PREC_FP32])
def test_gmres_batch_lens(prec):
    """n = 127 lens, 4 right-hand sides; each against its own oracle run."""
    n = 127
    w = workloads.workload("2d_n511_lens", n=n, nrhs=4)
    P = Problem.from_workload(w)
    with _plan(P, prec) as plan:
        u, it, rr, st = plan.gmres(dev(w["f"]), tol=1e-6, restart=20, maxit=200)
        u = host(u)
    assert st == asp.ASP_OK
    A = P.A()
    M = Preconditioner(P)
    for k in range(4):
        b = w["f"][k] / P.scale()
        x_ref, it_ref, _, _ = oracle_gmres(lambda v: A @ v, M.apply, b, 1e-6, 20, 200)
        assert abs(int(it[k]) - it_ref) <= 1
        assert np.linalg.norm(b - A @ u[k]) / np.linalg.norm(b) <= 1e-6 * (1 + 1e-9)
        assert rel(u[k], x_ref) < (1e-6 if prec == asp.ASP_PREC_FP64 else 1e-5)


def test_alone_equals_in_batch():
    """Each right-hand side gives bitwise the same result alone and in a batch."""
    w = workloads.workload("2d_n511_lens", n=95, nrhs=3)
    P = Problem.from_workload(w)
    with _plan(P, asp.ASP_PREC_FP32) as plan:
        u_all, it_all, _, _ = plan.gmres(dev(w["f"]), tol=1e-6, restart=20, maxit=100)
        u_all = host(u_all)
        for k in range(3):
            u1, it1, _, _ = plan.gmres(dev(w["f"][k:k + 1]), tol=1e-6, restart=20, maxit=100)
            assert int(it1[0]) == int(it_all[k])
            assert np.array_equal(host(u1)[0], u_all[k])


@pytest.mark.parametrize("prec,tol", [(asp.ASP_PREC_FP64, 1e-11), (asp.ASP_PREC_FP32, 8e-6)])
@pytest.mark.parametrize("n,gamma,b", [(63, 12, 4), (100, 12, 4), (127, 9, 8)])
def test_apply_sequential_sweep(n, gamma, b, prec, tol):
    """opts.sweep2d = ASP_SWEEP2D_SEQUENTIAL (Algorithm 2 as stated, no boundary
    maps): the apply against the oracle, and against the default path with
    the maps (the same operator, rounding apart)."""
    P = _problem(n, gamma, b)
    M = Preconditioner(P)
    rng = np.random.default_rng(4)
    r = rng.standard_normal((3, P.N)) + 1j * rng.standard_normal((3, P.N))
    with asp.Plan(2, P.c, P.omega, n, b, gamma, C=P.C, prec=prec,
                  sweep2d=asp.ASP_SWEEP2D_SEQUENTIAL) as plan:
        plan.factor()
        z = host(plan.apply(dev(r)))
    with _plan(P, prec) as plan:
        plan.factor()
        zm = host(plan.apply(dev(r)))
    for k in range(3):
        e = rel(z[k], M.apply(r[k]))
        print(f"2D sequential-sweep apply n={n} prec={prec}: rel err {e:.2e}, vs maps "
              f"{rel(z[k], zm[k]):.2e}", flush=True)
        assert e < tol
        assert rel(z[k], zm[k]) < (1e-12 if prec == asp.ASP_PREC_FP64 else 2 * tol)


def test_gmres_sequential_sweep_counts():
    """GMRES with the sequential sweeps takes the oracle's iteration counts."""
    w = workloads.workload("2d_n511_lens", n=127, nrhs=3)
    P = Problem.from_workload(w)
    with asp.Plan(2, w["c"], w["omega"], w["n"], w["b"], w["gamma"], C=w["C"],
                  sweep2d=asp.ASP_SWEEP2D_SEQUENTIAL) as plan:
        u, it, rr, st = plan.gmres(dev(w["f"]), tol=1e-6, restart=20, maxit=200)
        u = host(u)
    assert st == asp.ASP_OK
    A, M = P.A(), Preconditioner(P)
    for k in range(3):
        b = w["f"][k] / P.scale()
        x_ref, it_ref, _, _ = oracle_gmres(lambda v: A @ v, M.apply, b, 1e-6, 20, 200)
        assert abs(int(it[k]) - it_ref) <= 1
        assert rel(u[k], x_ref) < 1e-6


def test_gmres_long_cycle():
    """A hard case (2D n = 63, random velocity at 3 points per wavelength,
    GMRES(40) to 1e-10): the oracle needs 52 iterations, so one cycle runs
    past the 24 basis vectors of the fused Gram-Schmidt passes into the
    chunked ones, then restarts.  FP64 factors: the count within one of the
    oracle's, the true residual at the tolerance, the solution close."""
    n = 63
    w = workloads.workload("2d_n1023_random", n=n, nrhs=2)
    P = Problem(2, n, 2 * math.pi * (n + 1) / 3, 12, 25.0, 4, w["c"])
    A, M = P.A(), Preconditioner(P)
    with _plan(P) as plan:
        u, it, rr, st = plan.gmres(dev(w["f"]), tol=1e-10, restart=40, maxit=400)
        u = host(u)
    assert st == asp.ASP_OK
    for k in range(2):
        b = w["f"][k] / P.scale()
        x_ref, it_ref, _, _ = oracle_gmres(lambda v: A @ v, M.apply, b, 1e-10, 40, 400)
        e = rel(u[k], x_ref)
        print(f"long cycle rhs {k}: iters {int(it[k])} (oracle {it_ref}), error {e:.2e}", flush=True)
        assert it_ref > 40
        assert abs(int(it[k]) - it_ref) <= 1
        assert np.linalg.norm(b - A @ u[k]) / np.linalg.norm(b) <= 1e-10 * (1 + 1e-6)
        assert e < 1e-7
