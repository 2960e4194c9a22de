"""GPU parity of the nested-dissection path for the 3D auxiliary problems
(Section 4.1: columns along the sweep axis, ordered by nested dissection;
opts.nd3d) against the CPU FP64 oracle, through the C ABI: one auxiliary
Green's operator of each kind and the whole apply at FP64 (1e-11) and FP32
(1e-5 / 1e-5, about ten times the measured errors) factors, agreement with the dense block-recurrence path, more
than one chunk of 16 right-hand sides, and GMRES at the paper's 3D settings
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


# (n, gamma, b, gamma_aux): one to several tree levels, ragged regions, thin pads
CASES = [(9, 2, 2, None), (15, 4, 3, None), (23, 5, 4, 3), (26, 9, 3, 5)]


def _problem(n, gamma, b, aux, seed=3):
    c = workloads.velocity_random(n, 3, seed=seed, width=3.0)
    return Problem(3, n, 2 * math.pi * (n + 1) / 8, gamma, 25.0, b, c, gamma_aux=aux)


def _plan(P, prec, nd=True):
    return asp.Plan(3, P.c, P.omega, P.n, P.b, P.gamma, C=P.C, prec=prec,
                    pml_aux=P.gamma_aux, nd3d=nd)


# FP32: about ten times the largest measured error (1.0e-6 per operator)
@pytest.mark.parametrize("prec,tol", [(asp.ASP_PREC_FP64, 1e-11), (asp.ASP_PREC_FP32, 1e-5)])
@pytest.mark.parametrize("n,gamma,b,aux", CASES)
def test_nd_operators(n, gamma, b, aux, prec, tol):
    print(f"nd operators n={n} gamma={gamma} b={b} aux={aux} prec={prec}", flush=True)
    P = _problem(n, gamma, b, aux)
    X = partition.layers(n, b, gamma)
    subs = partition.subproblems(n, b, gamma, aux)
    m = len(X)
    picks = {"M": [1, 2, m], "R": [2, m], "L": [1, m - 1]}
    kinds = {"M": asp.ASP_SUB_M, "R": asp.ASP_SUB_R, "L": asp.ASP_SUB_L}
    rng = np.random.default_rng(17)
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
                    print(f"nd3d G~{kind}_{p} prec={prec}: rel err {e:.2e}", flush=True)
                    assert e < tol, (kind, p)


# FP32: about ten times the largest measured error (9.4e-7 per apply)
@pytest.mark.parametrize("prec,tol", [(asp.ASP_PREC_FP64, 1e-11), (asp.ASP_PREC_FP32, 1e-5)])
@pytest.mark.parametrize("n,gamma,b,aux", CASES)
def test_nd_apply(n, gamma, b, aux, prec, tol):
    print(f"nd apply n={n} gamma={gamma} b={b} aux={aux} prec={prec}", flush=True)
    P = _problem(n, gamma, b, aux)
    M = Preconditioner(P)
    rng = np.random.default_rng(9)
    r = rng.standard_normal((2, P.N)) + 1j * rng.standard_normal((2, P.N))
    with _plan(P, prec) as plan:
        plan.factor()
        z = host(plan.apply(dev(r)))
    for k in range(2):
        e = rel(z[k], M.apply(r[k]))
        print(f"nd3d apply prec={prec}: rel err {e:.2e}", flush=True)
        assert e < tol


def test_nd_matches_block_recurrence_and_chunks():
    """FP64: the nested-dissection apply equals the block-recurrence apply to
    rounding, for 20 right-hand sides (two chunks of 16, one partly used);
    each right-hand side also equals the oracle's."""
    print("nd vs block recurrence n=23, 20 rhs", flush=True)
    P = _problem(23, 5, 4, None, seed=5)
    rng = np.random.default_rng(21)
    r = rng.standard_normal((20, P.N)) + 1j * rng.standard_normal((20, P.N))
    with _plan(P, asp.ASP_PREC_FP64, nd=True) as plan:
        plan.factor()
        z_nd = host(plan.apply(dev(r)))
    with _plan(P, asp.ASP_PREC_FP64, nd=False) as plan:
        plan.factor()
        z_bl = host(plan.apply(dev(r)))
    assert rel(z_nd, z_bl) < 1e-12
    M = Preconditioner(P)
    for k in (0, 15, 16, 19):
        assert rel(z_nd[k], M.apply(r[k])) < 1e-11, k


@pytest.mark.parametrize("field", ["lens", "random"])
def test_nd_paper_gmres(field):
    """The paper's 3D settings (eta = 9h, eta_aux = 5h, b = 4, GMRES(40) to
    1e-3, point source and wave packet) at n = 23: the GPU count with nested
    dissection equals the oracle's within 1, true residual within the tolerance."""
    print(f"nd gmres paper3d {field} n=23", flush=True)
    w = workloads.paper_workload3d(field, 23)
    P = Problem.from_workload(w)
    A = P.A()
    M = Preconditioner(P)
    f = np.asarray(w["f"], dtype=np.complex128)
    refs = []
    for k in range(2):
        _, it_ref, _, _ = oracle_gmres(lambda v: A @ v, M.apply, f[k] / P.scale(), w["tol"],
                                       w["restart"], 100)
        refs.append(it_ref)
    with asp.Plan(3, w["c"], w["omega"], 23, w["b"], w["gamma"], C=w["C"], prec=asp.ASP_PREC_FP64,
                  pml_aux=w["gamma_aux"], nd3d=True) as plan:
        u, it, rres, st = plan.gmres(dev(f), tol=w["tol"], restart=w["restart"], maxit=100)
        u = host(u)
    assert st == asp.ASP_OK
    print(f"  gpu {[int(x) for x in it]} oracle {refs}", flush=True)
    for k in range(2):
        assert abs(int(it[k]) - refs[k]) <= 1
        bvec = f[k] / P.scale()
        assert np.linalg.norm(bvec - A @ u[k]) / np.linalg.norm(bvec) <= w["tol"] * (1 + 1e-9)


def test_nd_factorization_groups_match_block_recurrence():
    """3D n = 63 (gamma = 8, b = 4) in FP64: the nested-dissection fronts do
    not fit one factorization group (the problems are factored in two groups
    that share the level buffers), and the apply still equals the
    block-recurrence apply to rounding."""
    print("nd two groups vs block recurrence n=63 fp64", flush=True)
    n = 63
    c = workloads.velocity_lens3d(n)
    P = Problem(3, n, 2 * math.pi * (n + 1) / 8, 8, 25.0, 4, c)
    rng = np.random.default_rng(23)
    r = rng.standard_normal((2, P.N)) + 1j * rng.standard_normal((2, P.N))
    with _plan(P, asp.ASP_PREC_FP64, nd=True) as plan:
        plan.factor()
        z_nd = host(plan.apply(dev(r)))
    with _plan(P, asp.ASP_PREC_FP64, nd=False) as plan:
        plan.factor()
        z_bl = host(plan.apply(dev(r)))
    for k in range(2):
        assert rel(z_nd[k], z_bl[k]) < 1e-11, k
