"""GPU parity at the shape the benchmark runs, and the mixed-precision gate.

Shape.  The 2D benchmark solves 64 right-hand sides at gamma = 12, b = 4: the
M problems have L = 26 lines (32-row tiles, 32 right-hand sides per solve
workgroup, so two chunks per problem), the R/L problems L = 15 (16-row tiles,
64 per workgroup), and a sweep step takes 32 right-hand sides per RHS tile (two
tiles).  Here every one of those 64 right-hand sides is compared with the
oracle's Algorithm 2 apply at n = 255 (59 layers), and a 72-RHS batch adds a
second R/L chunk and a third, ragged M chunk and sweep tile.  Errors are
measured two ways: the relative 2-norm of each right-hand side, and per grid
line (fixed i2): the largest error on the line divided by the largest entry of
the oracle's vector, so that one wrong line cannot hide in a global norm.

Above 2^31 bytes of grid vectors (n = 1023 with more than 128 right-hand
sides) the layer solves write through plain stores instead of buffer
resources; a 129-RHS apply there must give bitwise the same vectors as the
same right-hand sides applied in batches of 64 (same kernels, buffer path).

Mixed precision (Algorithm 2 with FP32 layer factors and with bf16-split
products; Algorithm 4 with FP32 and with bf16-split Schur updates).  Two valid GMRES solutions at tol 1e-6 can
differ by up to cond(A) 1e-6, so the solution gate runs both sides to tol
1e-10 and then asks for a relative difference <= 1e-6 against the FP64
oracle's solution; at tol 1e-6 the iteration counts must be within one of the
oracle's, and the error reached there is printed."""
import functools
import math

import numpy as np
import pytest
import torch

import workloads
from oracle.gmres import gmres as oracle_gmres
from oracle.operator import Problem
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


def line_err(z, ref, n, d):
    """Per grid line of the sweep axis (the slowest index): the largest error
    on the line over the largest entry of ref; returns (worst, line index)."""
    S = n ** (d - 1)
    e = np.abs(np.asarray(z) - ref).reshape(n, S).max(axis=1) / np.abs(ref).max()
    k = int(np.argmax(e))
    return float(e[k]), k


HEAD_N, HEAD_GAMMA, HEAD_B = 255, 12, 4


@functools.lru_cache(maxsize=None)
def _headline():
    """The benchmark's recipe (random velocity, gamma 12, b 4, 8 points per
    wavelength) at n = 255, 72 seeded complex residuals and the oracle's
    applies of all of them."""
    w = workloads.workload("2d_n1023_random", n=HEAD_N, nrhs=1)
    P = Problem.from_workload(w)
    assert (P.gamma, P.b) == (HEAD_GAMMA, HEAD_B)
    M = Preconditioner(P)
    rng = np.random.default_rng(255)
    r = rng.standard_normal((72, P.N)) + 1j * rng.standard_normal((72, P.N))
    ref = np.stack([M.apply(x) for x in r])
    return w, P, r, ref


def _plan2d(w, prec):
    return asp.Plan(2, w["c"], w["omega"], w["n"], w["b"], w["gamma"], C=w["C"], prec=prec)


# FP32 bounds about ten times the measured worst case over the 64 right-hand
# sides (relative 2-norm 1.0e-6, worst line 1.3e-6)
@pytest.mark.parametrize("prec,tol,ltol", [(asp.ASP_PREC_FP64, 1e-11, 1e-11),
                                           (asp.ASP_PREC_FP32, 1e-5, 1.5e-5)])
def test_apply_64_rhs(prec, tol, ltol):
    """All 64 right-hand sides of the benchmark's batch shape against the
    oracle: two 32-RHS chunks per M problem, two 32-RHS sweep tiles."""
    print(f"headline apply n={HEAD_N} nrhs=64 prec={prec}", flush=True)
    w, P, r, ref = _headline()
    with _plan2d(w, prec) as plan:
        assert plan.info()["m"] == 59
        plan.factor()
        z = host(plan.apply(dev(r[:64])))
    errs = [rel(z[k], ref[k]) for k in range(64)]
    lerrs = [line_err(z[k], ref[k], P.n, 2) for k in range(64)]
    worst = max(range(64), key=lambda k: lerrs[k][0])
    print(f"  max rel {max(errs):.2e} (rhs {int(np.argmax(errs))}); worst line "
          f"{lerrs[worst][0]:.2e} (rhs {worst}, i2 = {lerrs[worst][1] + 1})", flush=True)
    for k in range(64):
        assert errs[k] < tol, (k, errs[k])
        assert lerrs[k][0] < ltol, (k, lerrs[k])


def test_apply_72_rhs_fp64():
    """72 right-hand sides: a second 64-RHS chunk of every R/L problem, a
    third (8-RHS) chunk of every M problem and a third, ragged sweep tile."""
    print(f"headline apply n={HEAD_N} nrhs=72 fp64", flush=True)
    w, P, r, ref = _headline()
    with _plan2d(w, asp.ASP_PREC_FP64) as plan:
        plan.factor()
        z = host(plan.apply(dev(r)))
    for k in range(72):
        assert rel(z[k], ref[k]) < 1e-11, k
        assert line_err(z[k], ref[k], P.n, 2)[0] < 1e-11, k


def test_apply_plain_store_path_bitwise():
    """n = 1023, FP64: 129 right-hand sides (16.9 MB each, 2.18 GB in all)
    take the plain-store output path of the layer solves; the result must
    equal, bitwise, the same right-hand sides applied as 64 + 64 + 1 (buffer
    stores, staged output lines)."""
    n, nrhs = 1023, 129
    print(f"plain-store path n={n} nrhs={nrhs} fp64", flush=True)
    assert nrhs * n * n * 16 >= 2 ** 31 and 64 * n * n * 16 < 2 ** 31
    w = workloads.workload("2d_n1023_random", nrhs=1)
    g = torch.Generator(device="cuda")
    g.manual_seed(1023)
    r = torch.randn(nrhs, n * n, dtype=torch.complex128, device="cuda", generator=g)
    with _plan2d(w, asp.ASP_PREC_FP64) as plan:
        plan.factor()
        parts = [plan.apply(r[a:b]) for a, b in ((0, 64), (64, 128), (128, 129))]
        z_parts = torch.cat(parts)
        z_all = plan.apply(r)
        torch.cuda.synchronize()
        assert torch.isfinite(torch.view_as_real(z_all)).all()
        assert torch.equal(z_all, z_parts)


# ---------------------------------------------------------------------------------
# mixed precision: the solution gate at tol 1e-10, iteration counts at tol 1e-6
# ---------------------------------------------------------------------------------
@functools.lru_cache(maxsize=None)
def _oracle_case(name, n, nrhs):
    w = workloads.workload(name, n=n, nrhs=nrhs)
    P = Problem.from_workload(w)
    A = P.A()
    M = Preconditioner(P)
    sols = {}
    for tol in (1e-6, 1e-10):
        out = []
        for k in range(nrhs):
            b = w["f"][k] / P.scale()
            x, it, rr, _ = oracle_gmres(lambda v: A @ v, M.apply, b, tol, w["restart"], 400)
            out.append((x, it, rr))
        sols[tol] = out
    return w, P, A, sols


def _gate(name, n, nrhs, prec, label, nd=True):
    w, P, A, sols = _oracle_case(name, n, nrhs)
    with asp.Plan(w["d"], w["c"], w["omega"], w["n"], w["b"], w["gamma"], C=w["C"], prec=prec,
                  nd3d=nd) as plan:
        f = dev(w["f"])
        u6, it6, rr6, st6 = plan.gmres(f, tol=1e-6, restart=w["restart"], maxit=400)
        u6 = host(u6)
        u10, it10, rr10, st10 = plan.gmres(f, tol=1e-10, restart=w["restart"], maxit=400)
        u10 = host(u10)
    assert st6 == asp.ASP_OK and st10 == asp.ASP_OK
    for k in range(nrhs):
        b = w["f"][k] / P.scale()
        x6, itr6, _ = sols[1e-6][k]
        x10, itr10, _ = sols[1e-10][k]
        e6, e10 = rel(u6[k], x6), rel(u10[k], x10)
        res10 = np.linalg.norm(b - A @ u10[k]) / np.linalg.norm(b)
        print(f"{label} rhs {k}: iters {int(it6[k])} (oracle {itr6}) at 1e-6, error vs oracle "
              f"{e6:.2e}; iters {int(it10[k])} (oracle {itr10}) at 1e-10, error {e10:.2e}, "
              f"relres {res10:.1e}", flush=True)
        assert abs(int(it6[k]) - itr6) <= 1
        assert np.linalg.norm(b - A @ u6[k]) / np.linalg.norm(b) <= 1e-6 * (1 + 1e-9)
        assert res10 <= 1e-10 * (1 + 1e-6)
        assert e10 <= 1e-6


@pytest.mark.parametrize("prec", [asp.ASP_PREC_FP32, asp.ASP_PREC_BF16X3], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("name,n,nrhs", [("2d_n511_lens", 127, 4), ("2d_n1023_random", 255, 4)])
def test_gate_2d(name, n, nrhs, prec):
    print(f"mixed-precision gate 2D {name} n={n} prec={prec}", flush=True)
    _gate(name, n, nrhs, prec, f"2D {name}@{n} prec={prec}")


@pytest.mark.parametrize("prec", [asp.ASP_PREC_FP32, asp.ASP_PREC_BF16X3], ids=["fp32", "bf16x3"])
def test_gate_3d(prec):
    print(f"mixed-precision gate 3D lens n=31 prec={prec}", flush=True)
    _gate("3d_n63_lens", 31, 2, prec, f"3D lens@31 prec={prec}")
