"""Served solves on the GPU: each request's result is the same alone and in the mix.

A seeded stream of 2D requests over several grids and velocity families runs
through the serving loop (factor cache, memory admission, continuous batching,
concurrent keys on their own streams).  Every request is then solved again on
its own, in a fresh plan, and must agree bitwise (solution and iteration
count); every served solve reaches the relative residual 1e-6, and one request
per key is checked against the CPU FP64 oracle."""
import numpy as np
import pytest
import torch

import workloads
from oracle.gmres import gmres as oracle_gmres
from oracle.operator import Problem
from oracle.sweep import Preconditioner

pytestmark = pytest.mark.gpu
asp = pytest.importorskip("paper_1504_04058_amd.asp")
serve = pytest.importorskip("paper_1504_04058_amd.serve")

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

SIZES = ((2, 31), (2, 47), (2, 63))


def _stream(count=24, rate=400.0):
    return workloads.request_stream(count=count, rate=rate, seed=11, sizes=SIZES, max_rhs=5)


def _alone(desc, prec):
    c, f = workloads.materialize(desc)
    with asp.Plan(desc["d"], c, desc["omega"], desc["n"], desc["b"], desc["gamma"],
                  prec=prec) as plan:
        plan.factor()
        u, it, rr, st = plan.gmres(torch.from_numpy(f).cuda(), tol=1e-6, restart=20, maxit=400)
        torch.cuda.synchronize()
        return u.cpu().numpy(), it, rr


@pytest.mark.parametrize("prec", [asp.ASP_PREC_FP32, asp.ASP_PREC_FP64])
def test_served_equals_alone(prec):
    descs = _stream()
    reqs = [serve.Request.from_description(d) for d in descs]
    backend = serve.AspBackend(prec=prec, tol=1e-6, restart=20, maxit=400)
    srv = serve.Server(backend, budget_bytes=8 << 30, max_rhs=16, workers=3)
    res, summ = srv.run(reqs)
    print(summ, flush=True)
    assert summ["completed"] == len(reqs), [r.status for r in res]
    assert summ["factorizations"] == len({d["key"] for d in descs})
    assert any(len(ids) > 1 for _, ids in srv.batches)      # some requests shared a solve
    for r in res:
        assert r.status == "ASP_OK" and np.all(r.relres <= 1e-6)
    for d, r in zip(descs, res):
        u1, it1, _ = _alone(d, prec)
        assert np.array_equal(it1, r.iters), d["rid"]
        assert np.array_equal(u1, r.u), d["rid"]


def test_served_matches_oracle():
    descs = _stream(count=10)
    reqs = [serve.Request.from_description(d) for d in descs]
    res, summ = serve.Server(serve.AspBackend(prec=asp.ASP_PREC_FP32), budget_bytes=8 << 30,
                             workers=2).run(reqs)
    assert summ["completed"] == len(reqs)
    checked = set()
    for d, r in zip(descs, res):
        if d["key"] in checked:
            continue
        checked.add(d["key"])
        c, f = workloads.materialize(d)
        P = Problem(2, d["n"], d["omega"], d["gamma"], 25.0, d["b"], c)
        A, M = P.A(), Preconditioner(P)
        b = f[0] / P.scale()
        x_ref, it_ref, _, _ = oracle_gmres(lambda v: A @ v, M.apply, b, 1e-6, 20, 400)
        assert abs(int(r.iters[0]) - it_ref) <= 1
        err = np.linalg.norm(r.u[0] - x_ref) / np.linalg.norm(x_ref)
        assert err < 1e-5, (d["rid"], err)


def test_tight_budget_evicts_and_stays_within_it():
    descs = _stream(count=16)
    reqs = [serve.Request.from_description(d) for d in descs]
    backend = serve.AspBackend(prec=asp.ASP_PREC_FP32)
    # room for about two resident plans of the largest grid plus one batch
    big = max(reqs, key=lambda r: r.n)
    budget = 2 * backend.factor_bytes(big) + backend.workspace_bytes(big, 16)
    srv = serve.Server(backend, budget_bytes=budget, max_rhs=16, workers=2)
    res, summ = srv.run(reqs)
    assert summ["completed"] == len(reqs)
    assert summ["peak_bytes"] <= budget
    assert summ["evictions"] > 0


def test_served_equals_alone_with_3d_keys():
    """A stream mixing 2D and 3D keys (3D n = 19, 23 by nested dissection):
    every request's solution and iteration count are bitwise the same as when
    it is solved alone in a fresh plan, and 3D keys run concurrently with 2D
    ones on their own streams."""
    descs = workloads.request_stream(count=16, rate=400.0, seed=13,
                                     sizes=((2, 31), (3, 19), (3, 23)), max_rhs=5)
    assert {d["d"] for d in descs} == {2, 3}
    reqs = [serve.Request.from_description(d) for d in descs]
    backend = serve.AspBackend(prec=asp.ASP_PREC_FP32, tol=1e-6, restart=20, maxit=400)
    srv = serve.Server(backend, budget_bytes=16 << 30, max_rhs=16, workers=3)
    res, summ = srv.run(reqs)
    print(summ, flush=True)
    assert summ["completed"] == len(reqs), [r.status for r in res]
    for r in res:
        assert r.status == "ASP_OK" and np.all(r.relres <= 1e-6)
    for d, r in zip(descs, res):
        u1, it1, _ = _alone(d, asp.ASP_PREC_FP32)
        assert np.array_equal(it1, r.iters), d["rid"]
        assert np.array_equal(u1, r.u), d["rid"]


def test_served_equals_alone_with_reused_memory():
    """The library's device-memory reuse (asp_set_cache_limit) under a budget
    that forces evictions, so that factors, work buffers and workspaces of one
    key land in blocks another key gave back: every request still agrees
    bitwise with its solve alone in a fresh plan; the kept bytes never exceed
    the limit and go back to the driver when the limit returns to 0."""
    descs = workloads.request_stream(count=20, rate=400.0, seed=17,
                                     sizes=((2, 47), (2, 63), (3, 19)), max_rhs=5)
    reqs = [serve.Request.from_description(d) for d in descs]
    limit = 1 << 30
    backend = serve.AspBackend(prec=asp.ASP_PREC_FP32, tol=1e-6, restart=20, maxit=400,
                               cache_bytes=limit)
    try:
        big = max(reqs, key=lambda r: r.n ** r.dim)
        budget = 2 * backend.factor_bytes(big) + backend.factor_work_bytes(big) + \
            backend.workspace_bytes(big, 16)
        srv = serve.Server(backend, budget_bytes=budget, max_rhs=16, workers=3)
        res, summ = srv.run(reqs)
        print(summ, "kept", asp.asp_cached_bytes(), flush=True)
        assert summ["completed"] == len(reqs), [r.status for r in res]
        assert summ["evictions"] > 0
        assert 0 < asp.asp_cached_bytes() <= limit
    finally:
        backend.close()
    assert asp.asp_cached_bytes() == 0
    for d, r in zip(descs, res):
        assert r.status == "ASP_OK" and np.all(r.relres <= 1e-6)
        u1, it1, _ = _alone(d, asp.ASP_PREC_FP32)
        assert np.array_equal(it1, r.iters), d["rid"]
        assert np.array_equal(u1, r.u), d["rid"]
