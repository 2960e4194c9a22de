"""Pins of oracle.subproblem: the banded LU against a dense solve, the
Dirichlet data term g = (-1/h^2)[w, 0, ..., 0] of Section 3.1 (PML on the sweep
sides only, as printed there), the solution of every auxiliary problem
satisfying the printed difference equation with the printed auxiliary PML
profile and the prescribed boundary values, H^M_1 = A when there is a single
layer, and the symmetry of G~^M."""
import itertools

import numpy as np
import pytest

from oracle import partition
from oracle.operator import Problem
from oracle.subproblem import Subproblem

C = 25.0
OMEGA = 2 * np.pi * 2.5


def printed_sigma(kind, p, t, gamma, b, m, eta):
    """sigma^M_q / sigma^R_p / sigma^L_p of Section 2.1 in grid units (n = 2 gamma + m b - 2)."""
    one = 2 * gamma + m * b - 1
    quad = lambda t0: (C / eta) * ((t - t0) / gamma) ** 2
    if kind == "M":
        lo_edge = gamma if p == 1 else gamma + (p - 1) * b
        hi_edge = one - gamma if p == m else gamma + p * b - 1
    elif kind == "R":
        lo_edge, hi_edge = gamma + (p - 1) * b - 1, gamma + p * b - 1
    else:
        lo_edge, hi_edge = gamma if p == 1 else gamma + (p - 1) * b, gamma + p * b
    if t < lo_edge:
        return quad(lo_edge)
    if t > hi_edge:
        return quad(hi_edge)
    return 0.0


def printed_residual(v_ext, c_ext, lo, n, gamma, sweep_s):
    """Printed eq. (2D)/(3D) (PML form on every axis, sweep axis last) applied to
    v_ext on the lines lo-1..hi+1, returned on lines lo..hi (paper form, not
    divided by s).  sweep_s(t) gives s on the sweep axis at grid coordinate t."""
    d = v_ext.ndim
    h = 1.0 / (n + 1)
    eta = gamma * h

    def s_cross(t):
        if t < gamma:
            sig = (C / eta) * ((t - gamma) / gamma) ** 2
        elif t <= n + 1 - gamma:
            sig = 0.0
        else:
            sig = (C / eta) * ((t - (n + 1 - gamma)) / gamma) ** 2
        return 1.0 / (1.0 + 1j * sig / OMEGA)

    L = v_ext.shape[-1] - 2
    out = np.zeros(v_ext.shape[:-1] + (L,), dtype=complex)
    for idx in itertools.product(*[range(k) for k in out.shape]):
        e = idx[:-1] + (idx[-1] + 1,)          # index into v_ext
        val = OMEGA ** 2 / c_ext[e] ** 2 * v_ext[e]
        for ax in range(d):
            up = list(e); up[ax] += 1
            dn = list(e); dn[ax] -= 1
            if ax == d - 1:
                t = lo + idx[-1]
                s0, sp_, sm = sweep_s(t), sweep_s(t + 0.5), sweep_s(t - 0.5)
                vu, vd = v_ext[tuple(up)], v_ext[tuple(dn)]
            else:
                t = idx[ax] + 1
                s0, sp_, sm = s_cross(t), s_cross(t + 0.5), s_cross(t - 0.5)
                vu = v_ext[tuple(up)] if t < n else 0.0
                vd = v_ext[tuple(dn)] if t > 1 else 0.0
            val += s0 / h * (sp_ / h * (vu - v_ext[e]) - sm / h * (v_ext[e] - vd))
        out[idx] = val
    return out


@pytest.mark.parametrize("d,gamma,b,m", [(2, 4, 3, 4), (3, 3, 2, 3), (1, 5, 3, 5)])
def test_auxiliary_solutions_satisfy_printed_problems(d, gamma, b, m):
    n = 2 * gamma + m * b - 2
    h = 1.0 / (n + 1)
    eta = gamma * h
    rng = np.random.default_rng(5)
    c = 0.8 + 0.4 * rng.random((n,) * d)
    P = Problem(d, n, OMEGA, gamma, C, b, c)
    X = partition.layers(n, b, gamma)
    subs = partition.subproblems(n, b, gamma)
    S = n ** (d - 1)
    for kind in ("M", "R", "L"):
        for sub in subs[kind]:
            sp_ = Subproblem(P, sub, X[sub.p - 1])
            L = sub.L
            shape = (n,) * (d - 1) + (L,)
            if kind == "M":
                y = rng.standard_normal(S * (X[sub.p - 1][1] - X[sub.p - 1][0] + 1)) + 0j
                g = np.zeros(S * L, dtype=complex)
                g[sp_._slice_of_lines(*X[sub.p - 1])] = y
                w = np.zeros(S, dtype=complex)
            else:
                w = rng.standard_normal(S) + 1j * rng.standard_normal(S)
                g = np.zeros(S * L, dtype=complex)
                blk = slice(0, S) if kind == "R" else slice(S * (L - 1), S * L)
                g[blk] = -sp_.boundary_coupling() * w
            v = sp_.solve(g)
            if kind == "M":
                np.testing.assert_allclose(sp_.G(y), sp_.restrict(v), rtol=0, atol=0)
            else:
                np.testing.assert_allclose(sp_.G(w), sp_.restrict(v), rtol=0, atol=0)
            # assemble v on lines lo-1 .. hi+1 with its Dirichlet values
            v_ext = np.zeros((n,) * (d - 1) + (L + 2,), dtype=complex)
            v_ext[..., 1:L + 1] = v.reshape(shape, order="F")
            wl = w.reshape((n,) * (d - 1), order="F") if d > 1 else w
            if kind == "R":
                v_ext[..., 0] = wl
            elif kind == "L":
                v_ext[..., L + 1] = wl
            lines = np.arange(sub.lo - 1, sub.hi + 2)
            c_ext = np.ones_like(v_ext, dtype=float)
            inner = c.reshape((n,) * d)[..., sub.lo - 1: sub.hi]
            c_ext[..., 1:L + 1] = inner
            sweep_s = lambda t: 1.0 / (1.0 + 1j * printed_sigma(kind, sub.p, t, gamma, b, m, eta) / OMEGA)
            res = printed_residual(v_ext, c_ext, sub.lo, n, gamma, sweep_s)
            # paper-form right-hand side: the symmetric-form g times prod s
            s_cross = P.axis[0]
            scale = np.array([sweep_s(t) for t in lines[1:-1]])
            prod = np.ones(shape, dtype=complex)
            for ax in range(d - 1):
                sh = [1] * d
                sh[ax] = n
                prod = prod * s_cross.reshape(sh)
            prod = prod * scale.reshape([1] * (d - 1) + [L])
            rhs = np.zeros(shape, dtype=complex)
            if kind == "M":
                rhs = (g.reshape(shape, order="F")) * prod
            scale_ref = np.abs(v).max() / h ** 2 + np.abs(rhs).max()
            np.testing.assert_allclose(res, rhs, rtol=0, atol=1e-10 * scale_ref,
                                       err_msg=f"{kind}{sub.p}")


@pytest.mark.parametrize("d", [2, 3])
def test_dirichlet_data_term_is_minus_w_over_h2(d):
    """With the PML on the sweep sides only (the setting of Sections 3.1, 4.1)
    the data term of H^R and H^L is exactly (-1/h^2) w."""
    n, gamma, b = (21, 4, 3) if d == 2 else (11, 3, 2)
    h = 1.0 / (n + 1)
    P = Problem(d, n, OMEGA, gamma, C, b, np.ones((n,) * d), pml_axes="sweep")
    X = partition.layers(n, b, gamma)
    subs = partition.subproblems(n, b, gamma)
    for sub in subs["R"] + subs["L"]:
        cp = Subproblem(P, sub, X[sub.p - 1], factor=False).boundary_coupling()
        np.testing.assert_allclose(cp, np.full(n ** (d - 1), 1.0 / h ** 2), rtol=1e-14)


def test_band_lu_matches_dense_and_single_layer_is_global():
    n, gamma, b = 21, 4, 3
    rng = np.random.default_rng(3)
    c = 0.8 + 0.4 * rng.random((n, n))
    P = Problem(2, n, OMEGA, gamma, C, b, c)
    X = partition.layers(n, b, gamma)
    for sub in partition.subproblems(n, b, gamma)["M"][:3]:
        sp_ = Subproblem(P, sub, X[sub.p - 1])
        g = rng.standard_normal(sp_.H.shape[0]) + 1j * rng.standard_normal(sp_.H.shape[0])
        np.testing.assert_allclose(sp_.solve(g), np.linalg.solve(sp_.H.toarray(), g),
                                   rtol=1e-11, atol=1e-14)
    # a single layer: H^M_1 is the global operator
    n1 = 2 * (gamma - 1) + 3
    P1 = Problem(2, n1, OMEGA, gamma, C, 5, np.ones((n1, n1)))
    (sub,) = partition.subproblems(n1, 5, gamma)["M"]
    H = Subproblem(P1, sub, (1, n1), factor=False).H
    assert abs(H - P1.A()).max() == 0.0


def test_GM_is_symmetric():
    """H^M_q = (H^M_q)^T, so the X_q x X_q block of its inverse (= G~^M_q) is symmetric."""
    n, gamma, b = 17, 4, 3
    P = Problem(2, n, OMEGA, gamma, C, b, 1.0 + 0.2 * np.random.default_rng(2).random((n, n)))
    X = partition.layers(n, b, gamma)
    sub = partition.subproblems(n, b, gamma)["M"][2]
    sp_ = Subproblem(P, sub, X[sub.p - 1])
    k = n * (X[sub.p - 1][1] - X[sub.p - 1][0] + 1)
    G = np.column_stack([sp_.G(np.eye(k)[:, j].astype(complex)) for j in range(k)])
    assert np.abs(G - G.T).max() <= 1e-12 * np.abs(G).max()
