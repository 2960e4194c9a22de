"""Pins of oracle.operator and oracle.direct: eq. (2D) / (3D) evaluated
pointwise as printed, the textbook Dirichlet-Laplacian spectrum when the PML
is switched off, exact complex symmetry of the symmetric form, and the direct
solve against a dense LAPACK solve (G = A^-1 = G^T)."""
import itertools

import numpy as np
import pytest

import workloads
from oracle import direct
from oracle.operator import Problem

OMEGA = 2 * np.pi * 3


def paper_s(t, n, gamma, C, omega):
    """s at x = t h from the printed sigma of Section 2 (grid units)."""
    h = 1.0 / (n + 1)
    eta = gamma * h
    if t < gamma:
        sig = (C / eta) * ((t - gamma) / gamma) ** 2
    elif t <= n + 1 - gamma:
        sig = 0.0
    else:
        sig = (C / eta) * ((t - (n + 1 - gamma)) / gamma) ** 2
    return 1.0 / (1.0 + 1j * sig / omega)


def paper_lhs(u, c, n, gamma, C, omega, pml_axes):
    """Left-hand side of eq. (2D) / eq. (3D) at every grid point, evaluated with
    loops exactly as printed: the PML operator s(x)/h (s(x+h/2)/h (u+ - u) -
    s(x-h/2)/h (u - u-)) along the sweep axis (the last one), and, along the
    other axes, the plain second difference (pml_axes="sweep", as printed) or
    the same PML form (pml_axes="all", the experiments' setting)."""
    d = u.ndim
    h = 1.0 / (n + 1)
    out = np.zeros_like(u)
    for idx in itertools.product(range(n), repeat=d):
        val = omega ** 2 / c[idx] ** 2 * u[idx]
        for ax in range(d):
            i = idx[ax] + 1   # 1-based line
            up = list(idx); up[ax] += 1
            dn = list(idx); dn[ax] -= 1
            u_up = u[tuple(up)] if i < n else 0.0
            u_dn = u[tuple(dn)] if i > 1 else 0.0
            if ax == d - 1 or pml_axes == "all":
                s0 = paper_s(i, n, gamma, C, omega)
                sp_ = paper_s(i + 0.5, n, gamma, C, omega)
                sm = paper_s(i - 0.5, n, gamma, C, omega)
                val += s0 / h * (sp_ / h * (u_up - u[idx]) - sm / h * (u[idx] - u_dn))
            else:
                val += (u_up - 2 * u[idx] + u_dn) / h ** 2
        out[idx] = val
    return out


@pytest.mark.parametrize("d,n,gamma", [(1, 21, 5), (2, 11, 4), (3, 7, 3)])
@pytest.mark.parametrize("pml_axes", ["sweep", "all"])
def test_symmetric_form_is_row_scaled_printed_equation(d, n, gamma, pml_axes):
    rng = np.random.default_rng(d * 100 + n)
    c = 0.8 + 0.4 * rng.random((n,) * d)
    P = Problem(d, n, OMEGA, gamma, 25.0, 3, c, pml_axes=pml_axes)
    u = rng.standard_normal((n,) * d) + 1j * rng.standard_normal((n,) * d)
    lhs = paper_lhs(u, c, n, gamma, 25.0, OMEGA, pml_axes)
    got = P.scale() * (P.A() @ workloads.flat(u))
    np.testing.assert_allclose(got, workloads.flat(lhs), rtol=1e-12, atol=1e-9 * np.abs(lhs).max())


@pytest.mark.parametrize("d,n", [(1, 30), (2, 12), (3, 6)])
def test_exact_complex_symmetry(d, n):
    rng = np.random.default_rng(7)
    c = 0.8 + 0.4 * rng.random((n,) * d)
    A = Problem(d, n, OMEGA, 3, 25.0, 2, c).A()
    assert abs(A - A.T).max() == 0.0


@pytest.mark.parametrize("d,n", [(1, 25), (2, 9), (3, 5)])
def test_sine_modes_without_pml(d, n):
    """C = 0 turns the PML off; the operator is then the Dirichlet Laplacian plus
    omega^2/c^2, whose eigenvectors are products of sines with eigenvalues
    -(4/h^2) sum_k sin^2(j_k pi h / 2) + omega^2/c^2."""
    h = 1.0 / (n + 1)
    A = Problem(d, n, OMEGA, 3, 0.0, 2, np.full((n,) * d, 1.3)).A()
    i = np.arange(1, n + 1)
    for modes in [(1,) * d, tuple(range(2, 2 + d)), (n,) * d]:
        vecs = [np.sin(j * np.pi * i * h) for j in modes]
        v = vecs[-1]
        for a in reversed(vecs[:-1]):
            v = np.kron(v, a)
        lam = -(4 / h ** 2) * sum(np.sin(j * np.pi * h / 2) ** 2 for j in modes) + OMEGA ** 2 / 1.3 ** 2
        np.testing.assert_allclose(A @ v, lam * v, rtol=0, atol=1e-9 * abs(lam))


@pytest.mark.parametrize("d,n", [(2, 9), (3, 5)])
def test_direct_solve_and_green_symmetry(d, n):
    rng = np.random.default_rng(11)
    c = 0.8 + 0.4 * rng.random((n,) * d)
    A = Problem(d, n, OMEGA, 3, 25.0, 2, c).A()
    b = rng.standard_normal(n ** d) + 1j * rng.standard_normal(n ** d)
    x = direct.solve(A, b)
    dense = np.asarray(A.todense())
    np.testing.assert_allclose(x, np.linalg.solve(dense, b), rtol=1e-11, atol=1e-13 * np.abs(x).max())
    G = direct.dense_inverse(A)
    assert np.abs(G - G.T).max() <= 1e-12 * np.abs(G).max()
