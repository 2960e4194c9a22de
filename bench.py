#!/usr/bin/env python3
"""Benchmark of the additive sweeping preconditioner inside GMRES on one MI355X.

A step is one pass of the whole hot path over one batch: factor every
auxiliary problem (Algorithm 1, plus the boundary maps of the sweeps) and solve
all right-hand sides of the batch with right-preconditioned GMRES(20) to
relative residual 1e-6 (Algorithm 2 applies, stencil applies, Arnoldi).  The
velocity field and sources are synthetic (workloads.py recipes) and resident
in device memory before the timed region.

Prints one JSON line (see the keys below).  `roofline` describes the kernel
class with the largest device time inside the timed region, measured with HIP
events around every launch by the library itself (asp_timing_*).
`cpu_baseline` times the CPU FP64 oracle on a bounded sample of the same
workload and scales it to solves/s.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Helmholtz solves/s to relres 1e-6 (2D n=1023, 3D n=63); PC-apply GB/s, MFMA%"

# MI355X published peaks.  Matrix cores: FP32 157.3, FP64 78.6 TFLOP/s (dense).
# Vector ALUs: 256 CUs x 64 lanes x 2 flops (FMA) x 2.4 GHz = 78.6 TFLOP/s for
# FP32 and FP64 alike; the 157.3 FP32 vector figure needs packed FP32
# instructions, which this build leaves off.
PEAK_HBM_GBS = 8000.0
PEAK_MFMA = {"fp32": 157.3, "fp64": 78.6, "bf16x3": 157.3}
PEAK_VALU = {"fp32": 78.6, "fp64": 78.6, "bf16x3": 78.6}

KCLASS = ["factor", "transfer", "solve_m", "solve_rl", "sweep", "combine", "stencil", "krylov"]
HBM_CLASSES = {"stencil", "krylov", "combine"}


def class_bound(dim, cls, prec):
    """(bound, peak, unit) of a kernel class: the layer solves, the boundary
    maps, the sweeps and the 3D factor run on the matrix cores; the 2D factor
    on the vector ALUs; stencil, Krylov and accumulation kernels stream HBM."""
    if cls in HBM_CLASSES:
        return "hbm", PEAK_HBM_GBS, "GB/s"
    if dim == 2 and cls == "factor":
        return "alu", PEAK_VALU[prec], "TFLOP/s"
    return "mfma", PEAK_MFMA[prec], "TFLOP/s"


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="2d_n1023_random")
    ap.add_argument("--prec", choices=["fp32", "fp64", "bf16x3"], default="fp32")
    ap.add_argument("--restart", type=int, default=None)
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain-fp64", action="store_true",
                    help="skip the plain FP64 lines beside a reduced-precision run")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only copy a device buffer of BYTES bytes once and exit: the "
                         "reference a hardware traffic counter is scaled by")
    ap.add_argument("--secondary", default="3d_n63_lens",
                    help="second workload timed after the first (same steps and warmup), '' for none")
    ap.add_argument("--serve-requests", type=int, default=48,
                    help="requests of the seeded serving stream timed after the batch runs (0: none)")
    ap.add_argument("--serve-spec", type=int, default=0, metavar="COUNT",
                    help="only run the full serving mix (2D n = 127..1023, 3D n = 31, 63, 1-32 "
                         "right-hand sides, half the requests repeating a key) of COUNT requests: "
                         "at saturation, then at fractions of the saturated request rate")
    ap.add_argument("--serve-fractions", default="0.5,0.8",
                    help="offered loads of --serve-spec as fractions of the saturated rate")
    ap.add_argument("--serve-sat-rate", type=float, default=0.0, metavar="REQ_PER_S",
                    help="with --serve-spec: skip the saturation run and take this saturated "
                         "request rate (from an earlier run) for the offered loads")
    ap.add_argument("--serve-budget-gb", type=float, default=200.0,
                    help="device memory the served factors and workspaces may hold")
    ap.add_argument("--cpu-sample", type=int, default=64,
                    help="auxiliary problems of each kind the oracle factors and solves")
    ap.add_argument("--paper-tables", default="",
                    help="comma-separated grid sizes of the paper's 2D experiments to run "
                         "(e.g. 127,255,511,1023,2047); '' for none")
    ap.add_argument("--paper-tables3d", default="",
                    help="grid sizes of the paper's 3D experiments to run (e.g. 39,79); '' for none")
    ap.add_argument("--paper-blocks3d", action="store_true",
                    help="factor the 3D paper tables by the dense block recurrence instead of "
                         "nested dissection")
    ap.add_argument("--sweep-compare", default="",
                    help="comma-separated 2D grid sizes: time the boundary-map sweeps against the "
                         "sequential R/L sweeps of Algorithm 2 (setup, one GMRES solve); '' for none")
    ap.add_argument("--paper-widths", default="",
                    help="NARROW:WIDE: run the 2D paper tables also with unequal layers of NARROW "
                         "or WIDE lines, wide where the velocity varies along the sweep axis "
                         "(workloads.variation_widths); '' for equal widths only")
    return ap.parse_args()


def prec_code(name):
    """The library's precision constant for a --prec name."""
    from paper_1504_04058_amd import asp

    return {"fp32": asp.ASP_PREC_FP32, "fp64": asp.ASP_PREC_FP64, "bf16x3": asp.ASP_PREC_BF16X3}[name]


def host_threads():
    """Threads of the host's CPU share: OMP_NUM_THREADS where the machine sets
    it (the GPU machines set their share there), else every core."""
    try:
        return max(1, int(os.environ.get("OMP_NUM_THREADS", "")))
    except ValueError:
        return os.cpu_count() or 1


def cpu_baseline(w, iters_mean, sample, threads=1):
    """Time the CPU FP64 oracle on a bounded sample of the workload and scale it
    to solves/s of the whole batch: factor `sample` auxiliary problems of each
    kind (M, R, L) and apply each G~ once; the full setup and one full
    preconditioner apply are the per-kind means times the counts; one solve of
    one right-hand side is then iters x (apply + stencil + Arnoldi), with the
    setup shared by the batch.  `threads`: BLAS/LAPACK threads (the oracle is
    one Python process; its banded LU and sparse matrix-vector products run in
    those libraries)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import partition
    from oracle.operator import Problem
    from oracle.subproblem import Subproblem

    with threadpool_limits(limits=threads):
        t_all = time.perf_counter()
        P = Problem.from_workload(w)
        X = partition.layers(P.n, P.b, P.gamma)
        subs = partition.subproblems(P.n, P.b, P.gamma)
        rng = np.random.default_rng(0)
        per_kind = {}
        for kind in ("M", "R", "L"):
            lst = subs[kind]
            picks = np.linspace(0, len(lst) - 1, min(sample, len(lst))).round().astype(int)
            tf = ts = 0.0
            for idx in sorted(set(picks.tolist())):
                s = lst[idx]
                t0 = time.perf_counter()
                sp = Subproblem(P, s, X[s.p - 1])
                t1 = time.perf_counter()
                k = P.S * (X[s.p - 1][1] - X[s.p - 1][0] + 1) if kind == "M" else P.S
                data = rng.standard_normal(k) + 1j * rng.standard_normal(k)
                sp.G(data)
                t2 = time.perf_counter()
                tf += t1 - t0
                ts += t2 - t1
            cnt = len(set(picks.tolist()))
            per_kind[kind] = (tf / cnt, ts / cnt, len(lst))
        A = P.A()
        v = rng.standard_normal(P.N) + 1j * rng.standard_normal(P.N)
        t0 = time.perf_counter()
        A @ v
        t_mv = time.perf_counter() - t0
        t0 = time.perf_counter()
        hv = np.vdot(v, v)
        t_dot = time.perf_counter() - t0
        t0 = time.perf_counter()
        v = v - hv * v
        t_axpy = time.perf_counter() - t0
        sample_s = time.perf_counter() - t_all
    setup = sum(f * c for f, _, c in per_kind.values())
    apply_ = sum(s * c for _, s, c in per_kind.values())
    # modified Gram-Schmidt at Arnoldi step j: j+1 dot products and updates
    arnoldi = (iters_mean / 2 + 1) * (t_dot + t_axpy)
    per_rhs = iters_mean * (apply_ + t_mv + arnoldi)
    nrhs = w["f"].shape[0]
    total = setup + nrhs * per_rhs
    return {
        "value": nrhs / total,
        "unit": "solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{sum(min(sample, c) for _, _, c in per_kind.values())} of "
                   f"{sum(c for _, _, c in per_kind.values())} auxiliary problems factored and "
                   f"solved once (banded LU, {threads} BLAS thread{'s' if threads > 1 else ''}) "
                   f"+ one stencil apply on the full grid, "
                   f"{sample_s:.1f} s; scaled by the problem counts and {iters_mean:.2f} GMRES "
                   f"iterations per RHS (the GPU run's mean), setup shared by {nrhs} RHS"),
        "setup_s": setup,
        "apply_s": apply_,
    }


def source_hash():
    """sha256 over the library's kernel and host sources (paper_1504_04058_amd/csrc)."""
    import hashlib

    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1504_04058_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".cpp", ".h")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(workload, prec_name, cls):
    """HBM bytes per launch of a kernel class from the committed counter record
    profiles/traffic_<workload>.md, or None when there is none for this
    workload, precision and class or the sources changed since it was taken."""
    import re

    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        m = re.search(r"<!-- traffic-json: (\{.*\}) -->", fh.read())
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("prec") != prec_name or rec.get("source_sha256") != source_hash():
        return None
    c = rec.get("classes", {}).get(cls)
    if not c:
        return None
    return c["fetch_bytes"] + c["write_bytes"]


def run_workload(name, prec_name, steps, warmup, restart=None, tol=None, nd3d=True, keep_u=False,
                 fact3d=None):
    """Time `steps` passes of the hot path (factor + GMRES of the whole batch)
    after `warmup` untimed passes; returns the measurements (and the last
    solution, on the device, if keep_u)."""
    import ctypes

    import torch

    import workloads
    from paper_1504_04058_amd import asp

    w = workloads.workload(name)
    restart = restart or w["restart"]
    tol = tol or w["tol"]
    prec = prec_code(prec_name)
    nrhs = w["f"].shape[0]
    dev = torch.device("cuda:0")
    f = torch.from_numpy(w["f"]).to(dev)
    u = torch.empty_like(f)
    plan = asp.Plan(w["d"], w["c"], w["omega"], w["n"], w["b"], w["gamma"], C=w["C"], prec=prec,
                    nd3d=nd3d, fact3d=fact3d)
    h = plan.handle
    L = asp.lib()
    for _ in range(warmup):
        asp.asp_factor(h)
        asp.asp_gmres(h, f, u, nrhs, tol, restart, 400)
    torch.cuda.synchronize()
    L.asp_timing_enable(h, 1)
    t_factor = t_gmres = 0.0
    results = []
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        asp.asp_factor(h)
        b = time.perf_counter()
        results.append(asp.asp_gmres(h, f, u, nrhs, tol, restart, 400))
        torch.cuda.synchronize()
        c = time.perf_counter()
        t_factor += b - a
        t_gmres += c - b
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.asp_timing_enable(h, 0)
    kstats = {}
    for ci, cname in enumerate(KCLASS):
        nl, ms, by, fl = ctypes.c_int(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        L.asp_timing_read(h, ci, ctypes.byref(nl), ctypes.byref(ms), ctypes.byref(by), ctypes.byref(fl))
        if nl.value:
            kstats[cname] = {"launches": nl.value, "ms": ms.value, "bytes": by.value, "flops": fl.value}
    info = plan.info()
    plan.close()
    st, iters, relres = results[-1]
    ms_step = (t1 - t0) * 1e3 / steps

    dom = max(kstats, key=lambda k: kstats[k]["ms"])
    ks = kstats[dom]
    bound, peak, unit = class_bound(w["d"], dom, prec_name)
    if bound == "hbm":
        achieved = ks["bytes"] / (ks["ms"] / 1e3) / 1e9
    else:
        achieved = ks["flops"] / (ks["ms"] / 1e3) / 1e12
    roof = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": recorded_traffic(name, prec_name, dom),
            "traffic_unit": "bytes per launch", "kernel_class": dom,
            "avg_launch_ms": ks["ms"] / ks["launches"], "launches": ks["launches"],
            "per_launch_bytes": ks["bytes"] / ks["launches"],
            "per_launch_flops": ks["flops"] / ks["launches"]}
    pc = [k for k in ("solve_m", "solve_rl", "sweep", "combine") if k in kstats]
    pc_ms = sum(kstats[k]["ms"] for k in pc)
    pc_bytes = sum(kstats[k]["bytes"] for k in pc)
    return {
        "w": w, "nrhs": nrhs, "restart": restart, "tol": tol,
        "value": nrhs / (ms_step / 1e3), "ms_per_step": ms_step,
        "warm_solves_per_s": nrhs / (t_gmres / steps),
        "factor_ms": t_factor * 1e3 / steps, "gmres_ms": t_gmres * 1e3 / steps,
        "iters": iters, "relres": relres, "status": asp.STATUS_NAMES.get(st, st),
        "pc_apply_gbps": pc_bytes / (pc_ms / 1e3) / 1e9 if pc_ms else None,
        "kernels": kstats, "roofline": roof, "factor_bytes": info["factor_bytes"],
        "u": u if keep_u else None,
    }


def serving_run(count, prec_name):
    """Served solves: a seeded stream of 2D (n = 127, 255, 511) and 3D (n = 31)
    requests, 1-8 right-hand sides each, half of them repeating an earlier
    problem, through the serving loop on a 64 GB device budget, all requests
    queued at the start (the loop's throughput, not the arrival rate)."""
    import workloads
    from paper_1504_04058_amd import asp, serve

    sizes = ((2, 127), (2, 255), (2, 511), (3, 31))
    descs = workloads.request_stream(count=count, rate=40.0, seed=5, sizes=sizes, max_rhs=8)
    reqs = []
    for d in descs:          # request payloads built before the stream starts
        c, f = workloads.materialize(d)
        reqs.append(serve.Request(d["rid"], d["key"], d["arrival"], d["d"], d["n"], d["omega"],
                                  d["nrhs"], c, f, layer_b=d["b"], pml_eta=d["gamma"]))
    prec = prec_code(prec_name)
    backend = serve.AspBackend(prec=prec, keep_u=False, cache_bytes=16 << 30)
    srv = serve.Server(backend, budget_bytes=64 << 30, max_rhs=64, workers=4, realtime=False)
    res, summ = srv.run(reqs)
    backend.close()
    summ["stream"] = {"requests": count, "arrivals": "all at the start", "seed": 5,
                      "sizes": [f"{d}d n={n}" for d, n in sizes], "rhs_per_request": "1-8",
                      "repeat": 0.5}
    summ["batches"] = len(srv.batches)
    summ["mean_batch_rhs"] = (sum(sum(reqs[i].nrhs for i in ids) for _, ids in srv.batches) /
                              max(len(srv.batches), 1))
    return summ


def serving_spec(prec_name, count, fractions, budget_gb, cache_gb=48.0, sat_rate=0.0):
    """The full serving mix: a seeded Poisson stream of `count` requests (2D
    n = 127, 255, 511, 1023 and 3D n = 31, 63 with omega = 2 pi n / 8; constant,
    lens and random velocities; 1-32 right-hand sides; each request repeats an
    earlier key with probability 1/2).  First all requests arrive at once (the
    saturated throughput and request rate), then the same stream arrives in
    real time at each fraction of the saturated request rate.  Requests build
    their inputs when they are served."""
    import workloads
    from paper_1504_04058_amd import asp, serve

    prec = prec_code(prec_name)
    budget = int(budget_gb * (1 << 30))

    def one(rate, realtime):
        descs = workloads.request_stream(count=count, rate=rate, seed=5, max_rhs=32)
        reqs = [serve.Request.from_description(d) for d in descs]
        backend = serve.AspBackend(prec=prec, keep_u=False, cache_bytes=int(cache_gb * (1 << 30)))
        srv = serve.Server(backend, budget_bytes=budget, max_rhs=64, workers=4, realtime=realtime,
                           progress_every=max(1, count // 10))
        res, summ = srv.run(reqs)
        backend.close()
        summ["offered_rate_per_s"] = rate if realtime else None
        summ["keys"] = len({d["key"] for d in descs})
        summ["batches"] = len(srv.batches)
        return summ

    if sat_rate > 0:
        sat = {"given_request_rate_per_s": sat_rate}
    else:
        print(f"serve-spec: {count} requests, saturation run", flush=True)
        sat = one(1.0, False)
        sat_rate = sat["completed"] / sat["wall_s"]
    out = {"stream": {"requests": count, "seed": 5, "sizes": "2D n = 127, 255, 511, 1023; 3D n = 31, 63",
                      "rhs_per_request": "1-32", "repeat": 0.5, "budget_gb": budget_gb,
                      "reuse_cache_gb": cache_gb,
                      "layer_precision": prec_name},
           "saturation": dict(sat, request_rate_per_s=sat_rate), "loads": []}
    for f in fractions:
        print(f"serve-spec: offered load {f:.2f} x {sat_rate:.2f} requests/s", flush=True)
        out["loads"].append(dict(one(f * sat_rate, True), fraction=f))
    return out


def sweep_compare(prec_name, sizes, nrhs=16):
    """The two 2D sweep forms side by side at each grid size (the
    2d_n1023_random recipe, 8 points per wavelength, nrhs right-hand sides,
    GMRES(20) to 1e-6): setup (a second factorization of the plan; the maps
    form computes its boundary maps there) and one GMRES solve (the second
    one), with the factor bytes of each form."""
    import torch

    import workloads
    from paper_1504_04058_amd import asp

    prec = prec_code(prec_name)
    rows = []
    for n in sizes:
        w = workloads.workload("2d_n1023_random", n=n, nrhs=nrhs)
        f = torch.from_numpy(w["f"]).cuda()
        u = torch.empty_like(f)
        for form, sw in (("maps", asp.ASP_SWEEP2D_MAPS), ("sequential", asp.ASP_SWEEP2D_SEQUENTIAL)):
            with asp.Plan(2, w["c"], w["omega"], n, w["b"], w["gamma"], C=w["C"], prec=prec,
                          sweep2d=sw) as plan:
                plan.factor()
                torch.cuda.synchronize()
                a = time.perf_counter()
                plan.factor()
                torch.cuda.synchronize()
                b = time.perf_counter()
                asp.asp_gmres(plan.handle, f, u, nrhs, 1e-6, 20, 200)
                torch.cuda.synchronize()
                c0 = time.perf_counter()
                st, iters, relres = asp.asp_gmres(plan.handle, f, u, nrhs, 1e-6, 20, 200)
                torch.cuda.synchronize()
                c = time.perf_counter()
                info = asp.asp_info(plan.handle)
            rows.append({"n": n, "form": form, "m": info["m"], "factor_bytes": info["factor_bytes"],
                         "setup_ms": (b - a) * 1e3, "solve_ms": (c - c0) * 1e3,
                         "iters_mean": float(iters.mean()), "max_relres": float(relres.max())})
            print(f"sweep-compare n={n} {form}: setup {rows[-1]['setup_ms']:.1f} ms, solve "
                  f"{rows[-1]['solve_ms']:.1f} ms", flush=True)
        del f, u
        torch.cuda.empty_cache()
    return {"workload": "2d_n1023_random recipe", "nrhs": nrhs, "layer_precision": prec_name,
            "rows": rows}


def paper_tables(prec_name, sizes, dim=2, widths=None, nd3d=True):
    """The paper's experiments (Tables 1-3 of Section 3.2 in 2D, Tables 4-6 of
    Section 4.2 in 3D) on this path: per field and grid, the factorization
    time (a second factorization of the plan; the first, which also allocates
    the factor memory, is reported beside it), the GMRES(40) iterations to 1e-3
    for force (a) point source and (b) wave packet (solved as one batch of two
    right-hand sides) and the solve time (again the second solve), beside the
    printed iteration counts.  widths = (narrow, wide): every
    problem once more with unequal layer widths from workloads.variation_widths."""
    import json as _json

    import torch

    import workloads
    from paper_1504_04058_amd import asp

    golden = "paper_iterations.json" if dim == 2 else "paper_iterations_3d.json"
    with open(os.path.join(ROOT, "tests", "golden", golden)) as fh:
        printed = _json.load(fh)
    prec = prec_code(prec_name)
    rows = []
    for n in sizes:
        col = printed["n"].index(n) if n in printed["n"] else None
        for field in workloads.PAPER_FIELDS:
            w = workloads.paper_workload(field, n) if dim == 2 else workloads.paper_workload3d(field, n)
            f = torch.from_numpy(w["f"]).cuda()
            u = torch.empty_like(f)
            layouts = [w["b"]]
            if widths:
                layouts.append(workloads.variation_widths(w["c"], w["gamma"], *widths))
            for lb in layouts:
                with asp.Plan(dim, w["c"], w["omega"], n, lb, w["gamma"], C=w["C"], prec=prec,
                              pml_aux=w.get("gamma_aux", 0), nd3d=nd3d and dim == 3) as plan:
                    torch.cuda.synchronize()
                    a0 = time.perf_counter()
                    plan.factor()   # first: includes allocating the factor and work memory
                    torch.cuda.synchronize()
                    a = time.perf_counter()
                    plan.factor()
                    torch.cuda.synchronize()
                    b = time.perf_counter()
                    st, iters, relres = asp.asp_gmres(plan.handle, f, u, 2, w["tol"], w["restart"],
                                                      200)
                    torch.cuda.synchronize()
                    c0 = time.perf_counter()
                    # again with the workspaces allocated: the steady-state solve time
                    st, iters, relres = asp.asp_gmres(plan.handle, f, u, 2, w["tol"], w["restart"],
                                                      200)
                    torch.cuda.synchronize()
                    c = time.perf_counter()
                    m = asp.asp_info(plan.handle)["m"]
                rows.append({"n": n, "omega_over_2pi": (n + 1) / 8, "field": field,
                             "layers": "equal" if isinstance(lb, int) else
                             f"variation {widths[0]}/{widths[1]}", "m": m,
                             "setup_ms": (b - a) * 1e3, "first_setup_ms": (a - a0) * 1e3,
                             "first_solve_ms": (c0 - b) * 1e3,
                             "solve_ms": (c - c0) * 1e3,
                             "iters": [int(i) for i in iters], "max_relres": float(max(relres)),
                             "status": asp.STATUS_NAMES.get(st, st),
                             "paper_iters": None if col is None else
                             [printed[field]["force_a"][col], printed[field]["force_b"][col]]})
            del f, u
            torch.cuda.empty_cache()
    settings = ("gamma 9, b 8, C 25, 8 points per wavelength, GMRES(40) to 1e-3, "
                "forces (a) point source at (1/2, 1/8), (b) wave packet at (1/8, 1/8)") if dim == 2 else \
               ("gamma 9, gamma_aux 5, b 4, C 25, 8 points per wavelength, GMRES(40) to 1e-3, "
                "forces (a) point source at (1/2, 1/2, 1/4), (b) wave packet at (1/2, 1/4, 1/4)")
    return {"settings": settings, "dim": dim, "layer_precision": prec_name, "rows": rows,
            "factorization": ("nested dissection" if nd3d else "block recurrence") if dim == 3 else None}


def workloads_dim(name):
    import workloads

    return workloads.WORKLOADS[name]["d"]


def config_of(name, r, prec_name):
    w = r["w"]
    return {"workload": name, "dim": w["d"], "n": w["n"], "nrhs": r["nrhs"],
            "omega_over_2pi": round(w["omega"] / (2 * math.pi), 6), "pml_eta": w["gamma"],
            "C": w["C"], "layer_b": w["b"], "restart": r["restart"], "tol": r["tol"],
            "layer_precision": prec_name, "krylov_precision": "fp64"}


def line_of(name, r, prec_name, factorization=None):
    """The measurements of one run_workload result as a bench sub-line."""
    cfg = config_of(name, r, prec_name)
    if factorization is not None:
        cfg["factorization"] = factorization
    return {
        "config": cfg, "value": r["value"], "unit": "solves/s", "ms_per_step": r["ms_per_step"],
        "warm_solves_per_s": r["warm_solves_per_s"], "factor_ms": r["factor_ms"],
        "gmres_ms": r["gmres_ms"], "iters_mean": float(r["iters"].mean()),
        "max_relres": float(r["relres"].max()), "status": r["status"],
        "pc_apply_gbps": r["pc_apply_gbps"], "kernels": r["kernels"], "roofline": r["roofline"],
    }


def compare_runs(mixed, plain):
    """Iterations per right-hand side of a reduced-precision run against the
    plain FP64 run of the same workload, and the relative 2-norm difference of
    their solutions (both to the same tolerance)."""
    import torch

    d = [int(a) - int(b) for a, b in zip(mixed["iters"], plain["iters"])]
    out = {"iter_delta": {"min": min(d), "max": max(d), "mean": sum(d) / len(d),
                          "rhs_differing": sum(1 for x in d if x != 0)}}
    if mixed.get("u") is not None and plain.get("u") is not None:
        um, up = mixed["u"], plain["u"]
        diff = torch.linalg.vector_norm(um - up, dim=1) / torch.linalg.vector_norm(up, dim=1)
        out["solution_rel_diff_max"] = float(diff.max())
    return out


def main():
    args = parse()
    if args.copy_probe:
        import torch

        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4}), flush=True)
        return
    if args.serve_spec:
        spec = serving_spec(args.prec, args.serve_spec,
                            [float(x) for x in args.serve_fractions.split(",")], args.serve_budget_gb,
                            sat_rate=args.serve_sat_rate)
        print(json.dumps({"serving_spec": spec}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU layout is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)
    r = run_workload(args.workload, args.prec, args.steps, args.warmup, args.restart, args.tol,
                     keep_u=args.prec != "fp64")
    iters, relres = r["iters"], r["relres"]
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": config_of(args.workload, r, args.prec),
        "warm_solves_per_s": r["warm_solves_per_s"],
        "factor_ms": r["factor_ms"],
        "gmres_ms": r["gmres_ms"],
        "iters": {"min": int(iters.min()), "max": int(iters.max()), "mean": float(iters.mean())},
        "max_relres": float(relres.max()),
        "status": r["status"],
        "pc_apply_gbps": r["pc_apply_gbps"],
        "kernels": r["kernels"],
        "roofline": r["roofline"],
        "cpu_baseline": None,
    }
    if args.prec != "fp64" and not args.no_plain_fp64:
        # the plain FP64 path on the same workload, and what the mixed path
        # changes against it: iterations per right-hand side and the solution
        p64 = run_workload(args.workload, "fp64", args.steps, args.warmup, args.restart, args.tol,
                           keep_u=True)
        out["plain_fp64"] = line_of(args.workload, p64, "fp64")
        out["plain_fp64"]["vs_mixed"] = compare_runs(r, p64)
        if args.prec != "bf16x3":
            # the same workload with real-split bf16 products in the layer
            # solves, boundary maps and sweeps (FP32 factors and accumulation)
            b16 = run_workload(args.workload, "bf16x3", args.steps, args.warmup, args.restart, args.tol,
                               keep_u=True)
            out["mixed_bf16x3"] = line_of(args.workload, b16, "bf16x3")
            out["mixed_bf16x3"]["vs_fp64"] = compare_runs(b16, p64)
            del b16
        del p64
    r["u"] = None
    if args.secondary:
        d2 = workloads_dim(args.secondary)
        from paper_1504_04058_amd import asp

        names = {asp.ASP_FACT3D_ND: "nested dissection", asp.ASP_FACT3D_BLOCKS: "block recurrence",
                 asp.ASP_FACT3D_RECURSIVE: "recursive sweep along x2"}
        for key, prec, f3 in (("secondary", args.prec, asp.ASP_FACT3D_ND),
                              ("secondary_bf16x3", "bf16x3", asp.ASP_FACT3D_ND),
                              ("secondary_blocks", args.prec, asp.ASP_FACT3D_BLOCKS),
                              ("secondary_recursive", args.prec, asp.ASP_FACT3D_RECURSIVE),
                              ("secondary_fp64", "fp64", asp.ASP_FACT3D_ND)):
            if (prec == "bf16x3" or f3 != asp.ASP_FACT3D_ND) and d2 != 3:
                continue
            if key == "secondary_fp64" and (args.prec == "fp64" or args.no_plain_fp64):
                continue
            s2 = run_workload(args.secondary, prec, args.steps, args.warmup, fact3d=f3 if d2 == 3 else None,
                              keep_u=key in ("secondary", "secondary_bf16x3", "secondary_fp64",
                                             "secondary_recursive"))
            out[key] = line_of(args.secondary, s2, prec, factorization=names[f3] if d2 == 3 else None)
            out[key]["_run"] = s2
        base = out.get("secondary_fp64", {}).get("_run")
        for key in ("secondary", "secondary_bf16x3", "secondary_recursive"):
            if base is not None and key in out:
                out[key]["vs_fp64"] = compare_runs(out[key]["_run"], base)
        for key in list(out):
            if isinstance(out[key], dict):
                out[key].pop("_run", None)
    if args.serve_requests > 0:
        out["serving"] = serving_run(args.serve_requests, args.prec)
    if args.paper_tables:
        out["paper_tables"] = paper_tables(args.prec, [int(x) for x in args.paper_tables.split(",")],
                                           widths=[int(x) for x in args.paper_widths.split(":")]
                                           if args.paper_widths else None)
    if args.sweep_compare:
        out["sweep_compare"] = sweep_compare(args.prec, [int(x) for x in args.sweep_compare.split(",")])
    if args.paper_tables3d:
        out["paper_tables3d"] = paper_tables(args.prec, [int(x) for x in args.paper_tables3d.split(",")],
                                             dim=3, nd3d=not args.paper_blocks3d)
    if not args.no_cpu_baseline:
        nt = host_threads()
        out["cpu_baseline"] = cpu_baseline(r["w"], float(iters.mean()), args.cpu_sample, threads=nt)
        if nt > 1:
            out["cpu_baseline"]["one_thread"] = cpu_baseline(r["w"], float(iters.mean()),
                                                             args.cpu_sample, threads=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
