"""asp_apply_noalloc (the apply for callers that cannot allocate) against
asp_apply: bitwise the same preconditioned vectors, on two calls in a row
with the second smaller than the first, in 2D (both precisions) and in 3D
(nested dissection); work buffers larger than the fixed array are refused with
an argument error before anything runs."""
import math

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu
asp = pytest.importorskip("paper_1504_04058_amd.asp")

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _inputs(nrhs, N, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return torch.randn(nrhs, N, dtype=torch.complex128, device="cuda", generator=g)


def _check_pair(plan, N, sizes, seed):
    for k, nrhs in enumerate(sizes):
        r = _inputs(nrhs, N, seed + k)
        z_ref = plan.apply(r)
        z = torch.full_like(r, float("nan"))
        plan.apply_noalloc(r, z)
        torch.cuda.synchronize()
        assert torch.isfinite(torch.view_as_real(z)).all()
        assert torch.equal(z, z_ref), (nrhs, float((z - z_ref).abs().max()))


@pytest.mark.parametrize("prec,sizes", [(asp.ASP_PREC_FP32, (5, 2)), (asp.ASP_PREC_FP64, (16, 3))])
def test_noalloc_2d(prec, sizes):
    print(f"noalloc 2D n=127 prec={prec} nrhs={sizes}", flush=True)
    w = workloads.workload("2d_n511_lens", n=127, nrhs=1)
    with asp.Plan(2, w["c"], w["omega"], 127, w["b"], w["gamma"], prec=prec) as plan:
        plan.factor()
        _check_pair(plan, 127 * 127, sizes, 11)


@pytest.mark.parametrize("n,gamma,prec,sizes", [(19, 4, asp.ASP_PREC_FP64, (3, 1)),
                                                 (31, 8, asp.ASP_PREC_FP32, (16, 5))])
def test_noalloc_3d(n, gamma, prec, sizes):
    print(f"noalloc 3D n={n} prec={prec} nrhs={sizes}", flush=True)
    c = workloads.velocity_lens3d(n)
    with asp.Plan(3, c, 2 * math.pi * (n + 1) / 8, n, 4, gamma, prec=prec) as plan:
        plan.factor()
        _check_pair(plan, n ** 3, sizes, 21)


def test_noalloc_refuses_oversized_work():
    print("noalloc oversized request", flush=True)
    w = workloads.workload("2d_n1023_random", n=255, nrhs=1)
    with asp.Plan(2, w["c"], w["omega"], 255, w["b"], w["gamma"], prec=asp.ASP_PREC_FP32) as plan:
        plan.factor()
        r = _inputs(64, 255 * 255, 3)
        z = torch.zeros_like(r)
        with pytest.raises(asp.AspError) as ei:
            plan.apply_noalloc(r, z)
        assert ei.value.status == asp.ASP_ERR_ARG and "scratch" in str(ei.value)
        torch.cuda.synchronize()
        assert not torch.any(z != 0)           # nothing ran
