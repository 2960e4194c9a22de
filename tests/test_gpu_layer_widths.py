"""GPU parity of unequal layer widths (Section 3.1 remarks: the layers need
not have the same width) against the CPU FP64 oracle, through the C ABI
(opts.n_layers / opts.layer_widths): one auxiliary Green's operator of each
kind, including a layer of a single line, and the whole apply, 2D and 3D, FP64
factors 1e-11 and FP32 factors 4e-5 / 3e-5 (about ten times the measured
errors); GMRES at the paper's 2D settings with wider layers across the lens,
with the oracle's iteration count."""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import partition
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


CASES = [(2, 40, 6, (3, 7, 1, 5, 6, 8)), (2, 63, 12, (1, 1, 9, 2, 4, 8, 8, 8)),
         (3, 23, 5, (1, 4, 2, 3, 5)), (3, 31, 8, (1, 4, 2, 3, 7))]


def _problem(d, n, gamma, w, seed=2):
    c = workloads.velocity_random(n, d, seed=seed, width=3.0 if d == 3 else 8.0)
    return Problem(d, n, 2 * math.pi * (n + 1) / 8, gamma, 25.0, list(w), c)


def _plan(P, prec):
    return asp.Plan(P.d, P.c, P.omega, P.n, list(P.b), P.gamma, C=P.C, prec=prec)


# FP32: about ten times the largest measured error (3.7e-6 per operator)
@pytest.mark.parametrize("prec,tol", [(asp.ASP_PREC_FP64, 1e-11), (asp.ASP_PREC_FP32, 4e-5)])
@pytest.mark.parametrize("d,n,gamma,w", CASES)
def test_unequal_width_operators(d, n, gamma, w, prec, tol):
    print(f"layer widths operators d={d} n={n} gamma={gamma} w={w} prec={prec}", flush=True)
    P = _problem(d, n, gamma, w)
    X = partition.layers(n, list(w), gamma)
    subs = partition.subproblems(n, list(w), gamma)
    m = len(X)
    one = [p for p in range(1, m + 1) if w[p - 1] == 1]
    picks = {"M": [1, 2, m] + one, "R": [2, m] + [p for p in one if p > 1],
             "L": [1, m - 1] + [p for p in one if p < m]}
    kinds = {"M": asp.ASP_SUB_M, "R": asp.ASP_SUB_R, "L": asp.ASP_SUB_L}
    rng = np.random.default_rng(13)
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
                    print(f"layer_widths G~{kind}_{p} prec={prec}: rel err {e:.2e}", flush=True)
                    assert e < tol, (kind, p)


# FP32: about ten times the largest measured error (3.1e-6 per apply)
@pytest.mark.parametrize("prec,tol", [(asp.ASP_PREC_FP64, 1e-11), (asp.ASP_PREC_FP32, 3e-5)])
@pytest.mark.parametrize("d,n,gamma,w", CASES)
def test_unequal_width_apply(d, n, gamma, w, prec, tol):
    print(f"layer widths apply d={d} n={n} w={w} prec={prec}", flush=True)
    P = _problem(d, n, gamma, w)
    M = Preconditioner(P)
    rng = np.random.default_rng(5)
    r = rng.standard_normal((3, P.N)) + 1j * rng.standard_normal((3, P.N))
    with _plan(P, prec) as plan:
        plan.factor()
        z = host(plan.apply(dev(r)))
    for k in range(3):
        e = rel(z[k], M.apply(r[k]))
        print(f"layer_widths apply prec={prec}: rel err {e:.2e}", flush=True)
        assert e < tol


def test_unequal_width_gmres_iterations():
    """2D paper settings at n = 127 (gamma = 9, 8 points per wavelength,
    GMRES(40) to 1e-3, both forces) with layers of 4 to 16 lines, wider
    across the lens: the GPU count equals the oracle's within 1."""
    w = workloads.paper_workload("lens", 127)
    widths = [4, 8, 16, 12, 16, 16, 8, 8, 4, 4, 6, 9]
    w["b"] = widths
    print(f"layer widths gmres n=127 w={widths}", flush=True)
    P = Problem.from_workload(w)
    A = P.A()
    M = Preconditioner(P)
    f = np.asarray(w["f"], dtype=np.complex128)
    refs = []
    for k in range(2):
        _, it_ref, rr, _ = oracle_gmres(lambda v: A @ v, M.apply, f[k] / P.scale(), w["tol"],
                                        w["restart"], 100)
        refs.append(it_ref)
    with _plan(P, asp.ASP_PREC_FP64) as plan:
        u, it, rres, st = plan.gmres(dev(f), tol=w["tol"], restart=w["restart"], maxit=100)
        u = host(u)
    assert st == asp.ASP_OK
    print(f"  gpu {[int(x) for x in it]} oracle {refs}", flush=True)
    for k in range(2):
        assert abs(int(it[k]) - refs[k]) <= 1
        bvec = f[k] / P.scale()
        assert np.linalg.norm(bvec - A @ u[k]) / np.linalg.norm(bvec) <= w["tol"] * (1 + 1e-9)


@pytest.mark.parametrize("d,n,gamma,aux,w", [(2, 63, 12, 4, (1, 1, 9, 2, 4, 8, 8, 8)),
                                             (3, 31, 8, 4, (1, 4, 2, 3, 7))])
def test_unequal_widths_with_thin_auxiliary_pml(d, n, gamma, aux, w):
    """Both options of the Section 3.1 remarks together: unequal layers and
    thinner auxiliary pads; the apply against the oracle in FP64."""
    print(f"layer widths + thin pml d={d} n={n} aux={aux} w={w}", flush=True)
    c = workloads.velocity_random(n, d, seed=4, width=3.0 if d == 3 else 8.0)
    P = Problem(d, n, 2 * math.pi * (n + 1) / 8, gamma, 25.0, list(w), c, gamma_aux=aux)
    M = Preconditioner(P)
    rng = np.random.default_rng(8)
    r = rng.standard_normal((2, P.N)) + 1j * rng.standard_normal((2, P.N))
    with asp.Plan(d, P.c, P.omega, n, list(w), gamma, C=P.C, prec=asp.ASP_PREC_FP64,
                  pml_aux=aux) as plan:
        plan.factor()
        z = host(plan.apply(dev(r)))
    for k in range(2):
        assert rel(z[k], M.apply(r[k])) < 1e-11


# 2D layers wider than 32 - 2 (gamma - 1) lines at gamma = 12: auxiliary
# problems of 33 to 64 lines run on blocks of 64 rows (FP64 up to 48 lines).
# Twenty right-hand sides: two workgroups of 16 per problem, the second ragged.
# Bounds about ten times the measured errors (FP32 1.4e-6 for operators and
# apply; bf16 split 1.7e-5 and 2.1e-5).
WIDE = [(asp.ASP_PREC_FP64, 1e-11, 1e-11, (26, 4, 20, 8, 26)),
        (asp.ASP_PREC_FP32, 1.5e-5, 1.5e-5, (40, 4, 30, 8, 42)),
        (asp.ASP_PREC_BF16X3, 2e-4, 2e-4, (40, 4, 30, 8, 42))]


@pytest.mark.parametrize("prec,tol_op,tol_apply,w", WIDE, ids=["fp64", "fp32", "bf16x3"])
def test_wide_layers_2d(prec, tol_op, tol_apply, w):
    gamma = 12
    n = sum(w) + 2 * (gamma - 1)
    print(f"wide layers 2D n={n} gamma={gamma} w={w} prec={prec}", flush=True)
    P = _problem(2, n, gamma, w)
    X = partition.layers(n, list(w), gamma)
    subs = partition.subproblems(n, list(w), gamma)
    m = len(X)
    kinds = {"M": asp.ASP_SUB_M, "R": asp.ASP_SUB_R, "L": asp.ASP_SUB_L}
    rng = np.random.default_rng(17)
    M = Preconditioner(P)
    r = rng.standard_normal((20, P.N)) + 1j * rng.standard_normal((20, P.N))
    with _plan(P, prec) as plan:
        plan.factor()
        for kind, ps in {"M": range(1, m + 1), "R": range(2, m + 1), "L": range(1, m)}.items():
            for p in ps:
                sub = [s for s in subs[kind] if s.p == p][0]
                ref = Subproblem(P, sub, X[p - 1])
                Np = P.S * (X[p - 1][1] - X[p - 1][0] + 1)
                k_in = Np if kind == "M" else P.S
                data = rng.standard_normal((2, k_in)) + 1j * rng.standard_normal((2, k_in))
                out = host(plan.subsolve(kinds[kind], p, dev(data), Np)).reshape(2, Np)
                for q in range(2):
                    e = rel(out[q], ref.G(data[q]))
                    print(f"wide G~{kind}_{p} (L={sub.L}) prec={prec}: rel err {e:.2e}", flush=True)
                    assert e < tol_op, (kind, p)
        z = host(plan.apply(dev(r)))
    worst = 0.0
    for k in range(20):
        worst = max(worst, rel(z[k], M.apply(r[k])))
    print(f"wide apply prec={prec}: max rel err {worst:.2e} over 20 right-hand sides", flush=True)
    assert worst < tol_apply
