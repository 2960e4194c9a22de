"""CPU tests of the C ABI: libasp.so loads and exports every function that
include/asp.h declares; the host-side partition and auxiliary grids equal the
oracle's bit for bit; the PML tables agree with the oracle to rounding; bad
arguments are rejected with ASP_ERR_ARG before any device work."""
import ctypes

import numpy as np
import pytest

from oracle import partition, pml

asp = pytest.importorskip("paper_1504_04058_amd.asp")


@pytest.fixture(scope="module")
def L():
    try:
        return asp.lib()
    except RuntimeError as e:   # not built
        pytest.fail(str(e))


def test_every_declared_symbol_is_exported(L):
    names = asp.declared_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(L, name), name


def _host_plan(dim, n, b, gamma, omega=2 * np.pi * 4, C=25.0):
    c = np.ones(n ** dim)
    return asp.asp_setup(dim, c, omega, n, b, gamma, C=C, host_only=True)


CONFIGS = [(2, 63, 4, 12), (2, 511, 4, 12), (2, 1023, 4, 12), (3, 63, 4, 8), (2, 127, 8, 9),
           (2, 2047, 8, 9), (3, 39, 4, 9), (2, 100, 4, 12), (2, 16, 8, 5), (2, 25, 4, 8),
           (2, 30, 3, 2), (3, 31, 4, 8)]


@pytest.mark.parametrize("dim,n,b,gamma", CONFIGS)
def test_partition_bit_exact(dim, n, b, gamma):
    plan = _host_plan(dim, n, b, gamma)
    try:
        layers, subs = asp.asp_layers(plan)
    finally:
        asp.asp_destroy(plan)
    X = partition.layers(n, b, gamma)
    assert [tuple(r) for r in layers.tolist()] == X
    ref = partition.subproblems(n, b, gamma)
    kinds = {"M": asp.ASP_SUB_M, "R": asp.ASP_SUB_R, "L": asp.ASP_SUB_L}
    want = [(kinds[k], s.p, s.lo, s.hi, s.phi, s.psi) for k in ("M", "R", "L") for s in ref[k]]
    assert [tuple(r) for r in subs.tolist()] == want


@pytest.mark.parametrize("dim,n,b,gamma", CONFIGS[:6])
def test_pml_tables_match_oracle(dim, n, b, gamma):
    omega = 2 * np.pi * (n + 1) / 8
    plan = _host_plan(dim, n, b, gamma, omega=omega)
    h = 1.0 / (n + 1)
    try:
        s_int, s_half = asp.asp_tables(plan, -1, n)
        ref_int, ref_half = pml.global_axis(n, 25.0, gamma, h, omega)
        np.testing.assert_allclose(s_int, ref_int, rtol=4e-16, atol=0)
        np.testing.assert_allclose(s_half, ref_half, rtol=4e-16, atol=0)
        _, subs = asp.asp_layers(plan)
        for k, (kind, p, lo, hi, phi, psi) in enumerate(subs.tolist()):
            s_int, s_half = asp.asp_tables(plan, k, hi - lo + 1)
            ref_int, ref_half = pml.tables(lo, hi, phi, psi, 25.0, gamma, h, omega)
            np.testing.assert_allclose(s_int, ref_int, rtol=4e-16, atol=0)
            np.testing.assert_allclose(s_half, ref_half, rtol=4e-16, atol=0)
    finally:
        asp.asp_destroy(plan)


AUX_CONFIGS = [(2, 127, 8, 9, 5), (3, 39, 4, 9, 5), (2, 63, 4, 12, 4), (2, 40, 5, 6, 2)]


@pytest.mark.parametrize("dim,n,b,gamma,aux", AUX_CONFIGS)
def test_thin_auxiliary_pml_matches_oracle(dim, n, b, gamma, aux):
    """pml_aux: the partition (bit-exact) and every sweep-axis table against
    the oracle's thin auxiliary pads (Section 3.1 remarks)."""
    omega = 2 * np.pi * (n + 1) / 8
    c = np.ones(n ** dim)
    plan = asp.asp_setup(dim, c, omega, n, b, gamma, host_only=True, pml_aux=aux)
    h = 1.0 / (n + 1)
    try:
        layers, subs = asp.asp_layers(plan)
        ref = partition.subproblems(n, b, gamma, aux)
        kinds = {"M": asp.ASP_SUB_M, "R": asp.ASP_SUB_R, "L": asp.ASP_SUB_L}
        refl = [s for k in ("M", "R", "L") for s in ref[k]]
        want = [(kinds[s.kind], s.p, s.lo, s.hi, s.phi, s.psi) for s in refl]
        assert [tuple(r) for r in subs.tolist()] == want
        for k, s in enumerate(refl):
            s_int, s_half = asp.asp_tables(plan, k, s.hi - s.lo + 1)
            ref_int, ref_half = pml.tables(s.lo, s.hi, s.phi, s.psi, 25.0, (s.gamma_lo, s.gamma_hi),
                                           h, omega)
            np.testing.assert_allclose(s_int, ref_int, rtol=4e-16, atol=0)
            np.testing.assert_allclose(s_half, ref_half, rtol=4e-16, atol=0)
    finally:
        asp.asp_destroy(plan)
    with pytest.raises(asp.AspError) as ei:
        asp.asp_setup(dim, c, omega, n, b, gamma, host_only=True, pml_aux=gamma + 1)
    assert ei.value.status == asp.ASP_ERR_ARG and "pml_aux" in str(ei.value)


WIDTH_CONFIGS = [(2, 40, 6, [3, 7, 1, 5, 6, 8]), (2, 127, 9, [4, 8, 16, 12, 16, 16, 8, 8, 4, 4, 6, 9]),
                 (3, 31, 8, [1, 4, 2, 3, 7]), (2, 63, 12, [1, 1, 9, 2, 4, 8, 8, 8]), (2, 30, 5, [22])]


@pytest.mark.parametrize("dim,n,gamma,w", WIDTH_CONFIGS)
def test_arbitrary_layer_widths_match_oracle(dim, n, gamma, w):
    """opts.n_layers / opts.layer_widths (Section 3.1 remarks: unequal layer
    widths): partition bit-exact with the oracle's, sweep-axis tables to
    rounding, and the planned factor bytes from the per-problem line counts."""
    omega = 2 * np.pi * (n + 1) / 8
    c = np.ones(n ** dim)
    plan = asp.asp_setup(dim, c, omega, n, w, gamma, host_only=True, prec=asp.ASP_PREC_FP32)
    h = 1.0 / (n + 1)
    try:
        layers, subs = asp.asp_layers(plan)
        assert [tuple(r) for r in layers.tolist()] == partition.layers(n, w, gamma)
        ref = partition.subproblems(n, w, gamma)
        kinds = {"M": asp.ASP_SUB_M, "R": asp.ASP_SUB_R, "L": asp.ASP_SUB_L}
        refl = [s for k in ("M", "R", "L") for s in ref[k]]
        assert [tuple(r) for r in subs.tolist()] == \
            [(kinds[s.kind], s.p, s.lo, s.hi, s.phi, s.psi) for s in refl]
        for k, s in enumerate(refl):
            s_int, s_half = asp.asp_tables(plan, k, s.hi - s.lo + 1)
            ref_int, ref_half = pml.tables(s.lo, s.hi, s.phi, s.psi, 25.0, gamma, h, omega)
            np.testing.assert_allclose(s_int, ref_int, rtol=4e-16, atol=0)
            np.testing.assert_allclose(s_half, ref_half, rtol=4e-16, atol=0)
        info = asp.asp_info(plan)
        assert info["m"] == len(w) and info["max_lines"] == max(s.L for s in refl)
        if dim == 2:
            m = len(w)
            want = 0
            for kind in [k for k in "MRL" if ref[k]]:
                group = ref["M"] if kind == "M" else ref["R"] + ref["L"]   # one row count per group
                LR = 16 if max(s.L for s in group) <= 16 else 32
                for s in ref[kind]:
                    # map problems: the map (rows padded to 16) and two columns
                    # of each diagonal block of H^-1
                    want += n * s.L * LR + ((-(-n // 16) * 16 + 2 * LR) * n
                                            if kind != "M" and 1 < s.p < m else 0)
            assert info["factor_bytes"] == want * 8
    finally:
        asp.asp_destroy(plan)


@pytest.mark.parametrize("w,frag", [([3, 7, 1, 5, 6, 7], "sum"), ([3, 0, 28], ">= 1"),
                                    ([31, -1], ">= 1"), ([60, 3], "sweep lines")])
def test_bad_layer_widths_rejected(L, w, frag):
    n, gamma = 40 if frag != "sweep lines" else 73, 6
    with pytest.raises(asp.AspError) as ei:
        asp.asp_setup(2, np.ones(n * n), 10.0, n, w, gamma, host_only=True)
    assert ei.value.status == asp.ASP_ERR_ARG and frag in str(ei.value)


@pytest.mark.parametrize("args,frag", [
    ((4, 63, 4, 12), "dim"),
    ((2, 20, 4, 12), "n too small"),
    ((2, 63, 0, 12), "layer_b"),
    ((2, 63, 4, 1), "pml_eta"),
    ((2, 127, 50, 12), "sweep lines"),
])
def test_bad_arguments_rejected(L, args, frag):
    dim, n, b, gamma = args
    with pytest.raises(asp.AspError) as ei:
        asp.asp_setup(dim, np.ones(max(n, 1) ** min(dim, 3)), 10.0, n, b, gamma, host_only=True)
    assert ei.value.status == asp.ASP_ERR_ARG and frag in str(ei.value)


def test_wide_2d_layers(L):
    """2D auxiliary problems of 33 to 64 lines take blocks of 64 rows; FP64
    plans stop at 48 lines, FP32 and bf16-split plans at 64."""
    gamma = 12
    for w, ok64, ok32 in (((26, 4, 20, 8, 26), True, True), ((27, 4, 20), False, True),
                          ((42, 4, 30), False, True), ((43, 4), False, False)):
        n = sum(w) + 2 * (gamma - 1)
        for prec, ok in ((asp.ASP_PREC_FP64, ok64), (asp.ASP_PREC_FP32, ok32),
                         (asp.ASP_PREC_BF16X3, ok32)):
            if not ok:
                with pytest.raises(asp.AspError) as ei:
                    asp.asp_setup(2, np.ones(n * n), 10.0, n, list(w), gamma, prec=prec, host_only=True)
                assert ei.value.status == asp.ASP_ERR_ARG and "sweep lines" in str(ei.value)
                continue
            plan = asp.asp_setup(2, np.ones(n * n), 10.0, n, list(w), gamma, prec=prec, host_only=True)
            try:
                info = asp.asp_info(plan)
                assert info["max_lines"] == max(w) + 2 * (gamma - 1)
                lay = asp.asp_layers(plan)
                # factor: n blocks of L x 64 per problem (every problem of a kind
                # shares the row count of its widest member), plus the maps
                ref = partition.subproblems(n, list(w), gamma)
                m = len(w)
                want = 0
                for kind in ("M", "R", "L"):
                    LR = max(16 if s.L <= 16 else 32 if s.L <= 32 else 64
                             for s in (ref["M"] if kind == "M" else ref["R"] + ref["L"]))
                    for s in ref[kind]:
                        want += n * s.L * LR + ((-(-n // 16) * 16 + 2 * LR) * n
                                                if kind != "M" and 1 < s.p < m else 0)
                esz = 16 if prec == asp.ASP_PREC_FP64 else 8
                assert info["factor_bytes"] == want * esz
                assert lay is not None
            finally:
                asp.asp_destroy(plan)


def test_bad_velocity_and_omega(L):
    c = np.ones(63 * 63)
    c[100] = np.nan
    with pytest.raises(asp.AspError) as ei:
        asp.asp_setup(2, c, 10.0, 63, 4, 12, host_only=True)
    assert ei.value.status == asp.ASP_ERR_ARG
    with pytest.raises(asp.AspError):
        asp.asp_setup(2, np.ones(63 * 63), -1.0, 63, 4, 12, host_only=True)
    c = np.ones(63 * 63)
    c[5] = 0.0
    with pytest.raises(asp.AspError):
        asp.asp_setup(2, c, 10.0, 63, 4, 12, host_only=True)


def test_host_only_plan_refuses_device_calls(L):
    plan = _host_plan(2, 63, 4, 12)
    try:
        assert L.asp_factor(plan) == asp.ASP_ERR_STATE
        assert L.asp_apply(plan, ctypes.c_void_p(16), ctypes.c_void_p(32), 1) == asp.ASP_ERR_STATE
        assert L.asp_matvec(plan, ctypes.c_void_p(16), ctypes.c_void_p(32), 1) == asp.ASP_ERR_STATE
        info = asp.asp_info(plan)
        assert info["m"] == 11 and info["n_sub"] == 31 and info["max_lines"] == 26
        assert "host-only" in asp.asp_last_error(plan)
        # null and aliasing pointers are argument errors
        assert L.asp_apply(plan, None, None, 1) == asp.ASP_ERR_ARG
    finally:
        asp.asp_destroy(plan)


def test_empty_and_bad_solve_arguments_rejected(L):
    """Zero or negative right-hand-side counts, bad GMRES controls and
    out-of-range auxiliary problems are argument errors, caught before the
    plan's state or the device is looked at (a host-only plan)."""
    plan = _host_plan(2, 63, 4, 12)
    a, b = ctypes.c_void_p(16), ctypes.c_void_p(32)
    it = (ctypes.c_int * 2)()
    rr = (ctypes.c_double * 2)()
    try:
        for nrhs in (0, -1):
            assert L.asp_apply(plan, a, b, nrhs) == asp.ASP_ERR_ARG
            assert L.asp_matvec(plan, a, b, nrhs) == asp.ASP_ERR_ARG
            assert L.asp_subsolve(plan, asp.ASP_SUB_M, 1, a, b, nrhs) == asp.ASP_ERR_ARG
            assert L.asp_gmres(plan, a, b, nrhs, 1e-6, 20, 100, it, rr) == asp.ASP_ERR_ARG
        assert L.asp_apply(plan, a, a, 1) == asp.ASP_ERR_ARG                # aliasing
        assert L.asp_gmres(plan, a, a, 1, 1e-6, 20, 100, it, rr) == asp.ASP_ERR_ARG
        for tol, restart, maxit in ((0.0, 20, 100), (-1e-6, 20, 100), (float("nan"), 20, 100),
                                    (1e-6, 0, 100), (1e-6, 65, 100), (1e-6, 20, 0)):
            assert L.asp_gmres(plan, a, b, 1, tol, restart, maxit, it, rr) == asp.ASP_ERR_ARG
        assert L.asp_gmres(plan, a, b, 1, 1e-6, 20, 100, None, rr) == asp.ASP_ERR_ARG
        m = asp.asp_info(plan)["m"]
        # G~^M_p for p = 1..m, G~^R_p for p = 2..m, G~^L_p for p = 1..m-1
        for kind, p in ((asp.ASP_SUB_M, 0), (asp.ASP_SUB_M, m + 1), (asp.ASP_SUB_R, 1),
                        (asp.ASP_SUB_L, m), (7, 1)):
            assert L.asp_subsolve(plan, kind, p, a, b, 1) == asp.ASP_ERR_ARG
    finally:
        asp.asp_destroy(plan)


@pytest.mark.parametrize("dim,n,b,gamma,prec", [(2, 1023, 4, 12, 1), (2, 63, 4, 12, 0),
                                                (3, 63, 4, 8, 1), (3, 31, 4, 8, 0)])
def test_planned_factor_bytes(dim, n, b, gamma, prec):
    """The planned factor size: 2D, n blocks of L x LR per problem (LR = 16 or
    32 rows) plus, for R_p and L_p with 1 < p < m, an n x n boundary map and
    two columns of each of the n diagonal blocks of H^-1; 3D with the
    block recurrence, n dense blocks of B x B with B = n L rounded up to a
    multiple of 64."""
    c = np.ones(n ** dim)
    plan = asp.asp_setup(dim, c, 2 * np.pi * 4, n, b, gamma, prec=prec, host_only=True, nd3d=False)
    try:
        info = asp.asp_info(plan)
    finally:
        asp.asp_destroy(plan)
    esz = 8 if prec == 1 else 16
    subs = partition.subproblems(n, b, gamma)
    m = len(partition.layers(n, b, gamma))
    want = 0
    for kind in ("M", "R", "L"):
        Ls = [s.hi - s.lo + 1 for s in subs[kind]]
        for s, L in zip(subs[kind], Ls):
            if dim == 2:
                LR = 16 if max(Ls) <= 16 else 32
                want += n * L * LR
                if kind != "M" and 1 < s.p < m:
                    want += -(-n // 16) * 16 * n     # boundary map, rows padded to 16
                    want += 2 * LR * n               # two columns of each diagonal block of H^-1
            else:
                B = -(-n * L // 64) * 64
                want += n * B * B
    assert info["factor_bytes"] == want * esz
    assert info["factored"] == 0
    if dim == 3 and n == 63 and prec == 1:
        assert 13.9e9 < info["factor_bytes"] < 15.0e9     # 13.9 GB unpadded, ~3% padding


@pytest.mark.parametrize("n,b,gamma,aux", [(63, 4, 8, 0), (79, 4, 9, 5), (39, 4, 9, 5)])
def test_nested_dissection_plan(L, n, b, gamma, aux):
    """opts.fact3d (Section 4.1): nested dissection (the default) has the same
    partition and fewer factor entries than the dense x1-blocks at these
    sizes; 2D plans ignore the field; unknown values are rejected."""
    c = np.ones(n ** 3)
    nd = asp.asp_setup(3, c, 10.0, n, b, gamma, host_only=True, pml_aux=aux,
                       prec=asp.ASP_PREC_FP32)
    dense = asp.asp_setup(3, c, 10.0, n, b, gamma, host_only=True, pml_aux=aux, nd3d=False,
                          prec=asp.ASP_PREC_FP32)
    try:
        a, b_ = asp.asp_info(nd), asp.asp_info(dense)
        assert a["m"] == b_["m"] and a["n_sub"] == b_["n_sub"]
        assert 0 < a["factor_bytes"] < b_["factor_bytes"]
        assert [tuple(r) for r in asp.asp_layers(nd)[1].tolist()] == \
            [tuple(r) for r in asp.asp_layers(dense)[1].tolist()]
    finally:
        asp.asp_destroy(nd)
        asp.asp_destroy(dense)
    for flag in (True, False):
        p2 = asp.asp_setup(2, np.ones(63 * 63), 10.0, 63, 4, 12, host_only=True, nd3d=flag)
        asp.asp_destroy(p2)
    opts = asp.asp_opts(25.0, asp.ASP_PREC_FP64, None, 1, 0, 0, None, 7)
    plan = ctypes.c_void_p()
    st = L.asp_setup(ctypes.byref(plan), 3, c.ctypes.data_as(ctypes.c_void_p), ctypes.c_double(10.0),
                     n, b, gamma, ctypes.byref(opts))
    assert st == asp.ASP_ERR_ARG and "fact3d" in asp.asp_last_error(plan)
    asp.asp_destroy(plan)


def test_bf16_split_precision_storage(L):
    """ASP_PREC_BF16X3 keeps FP32 factors (the split happens in the products),
    in 2D and 3D alike."""
    for dim, n, gamma in ((2, 63, 12), (3, 31, 8)):
        c = np.ones(n ** dim)
        plan = asp.asp_setup(dim, c, 10.0, n, 4, gamma, prec=asp.ASP_PREC_BF16X3, host_only=True)
        try:
            fp32 = asp.asp_setup(dim, c, 10.0, n, 4, gamma, prec=asp.ASP_PREC_FP32, host_only=True)
            try:
                assert asp.asp_info(plan)["factor_bytes"] == asp.asp_info(fp32)["factor_bytes"]
            finally:
                asp.asp_destroy(fp32)
        finally:
            asp.asp_destroy(plan)


def test_sequential_sweep_plan(L):
    """opts.sweep2d (Algorithm 2 as stated): the same partition and layer
    factors as the default, without the n x n boundary maps and the columns of
    the diagonal blocks of H^-1 they are built from; 3D plans ignore
    the field; unknown values are rejected."""
    n, b, gamma = 255, 4, 12
    c = np.ones(n * n)
    maps = asp.asp_setup(2, c, 10.0, n, b, gamma, host_only=True, prec=asp.ASP_PREC_FP32)
    seq = asp.asp_setup(2, c, 10.0, n, b, gamma, host_only=True, prec=asp.ASP_PREC_FP32,
                        sweep2d=asp.ASP_SWEEP2D_SEQUENTIAL)
    try:
        a, s_ = asp.asp_info(maps), asp.asp_info(seq)
        m = a["m"]
        assert s_["m"] == m and s_["n_sub"] == a["n_sub"]
        subs = partition.subproblems(n, b, gamma)
        lr_rl = 16 if max(sb.L for k in "RL" for sb in subs[k]) <= 16 else 32
        assert a["factor_bytes"] - s_["factor_bytes"] == \
            2 * (m - 2) * ((-(-n // 16) * 16) + 2 * lr_rl) * n * 8
    finally:
        asp.asp_destroy(maps)
        asp.asp_destroy(seq)
    p3 = asp.asp_setup(3, np.ones(23 ** 3), 10.0, 23, 4, 8, host_only=True,
                       sweep2d=asp.ASP_SWEEP2D_SEQUENTIAL)
    asp.asp_destroy(p3)
    opts = asp.asp_opts(25.0, asp.ASP_PREC_FP64, None, 1, 0, 0, None, 0, 5)
    plan = ctypes.c_void_p()
    st = L.asp_setup(ctypes.byref(plan), 2, c.ctypes.data_as(ctypes.c_void_p), ctypes.c_double(10.0),
                     n, b, gamma, ctypes.byref(opts))
    assert st == asp.ASP_ERR_ARG and "sweep2d" in asp.asp_last_error(plan)
    asp.asp_destroy(plan)


def test_recursive_plan(L):
    """opts.fact3d = ASP_FACT3D_RECURSIVE (Section 5): (3m-2)^2 inner problems,
    inner problem (outer o, inner i) factored as n blocks of B x B with B =
    L_o L_i rounded up to a multiple of 64; unequal layer widths are refused."""
    n, b, gamma = 31, 4, 8
    c = np.ones(n ** 3)
    plan = asp.asp_setup(3, c, 10.0, n, b, gamma, host_only=True, prec=asp.ASP_PREC_FP32,
                         fact3d=asp.ASP_FACT3D_RECURSIVE)
    try:
        info = asp.asp_info(plan)
    finally:
        asp.asp_destroy(plan)
    subs = partition.subproblems(n, b, gamma)
    Ls = [s.L for k in ("M", "R", "L") for s in subs[k]]
    want = sum(n * (-(-lo * li // 64) * 64) ** 2 for lo in Ls for li in Ls)
    assert info["factor_bytes"] == want * 8 and info["n_sub"] == len(Ls)
    with pytest.raises(asp.AspError) as e:
        asp.asp_setup(3, c, 10.0, n, [5, 5, 7], gamma, host_only=True,
                      fact3d=asp.ASP_FACT3D_RECURSIVE)
    assert e.value.status == asp.ASP_ERR_ARG and "equal layer widths" in str(e.value)
