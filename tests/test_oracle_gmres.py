"""Pins of oracle.gmres: after k steps the unpreconditioned iterate is the
least-squares minimiser of ||b - A x|| over the Krylov space K_k(A, b)
(computed here independently with numpy's QR and lstsq); exact
preconditioning converges in one step; restarted runs reach the direct
solution; residual estimates never increase inside a cycle."""
import numpy as np
import pytest

from oracle import direct
from oracle.gmres import gmres
from oracle.operator import Problem


def _system(n=12, omega=2 * np.pi * 2, C=25.0):
    rng = np.random.default_rng(9)
    P = Problem(2, n, omega, 3, C, 3, 0.9 + 0.2 * rng.random((n, n)))
    A = P.A()
    b = rng.standard_normal(P.N) + 1j * rng.standard_normal(P.N)
    return A, b


@pytest.mark.parametrize("k", [1, 3, 7])
def test_krylov_least_squares(k):
    A, b = _system()
    x, it, _, hist = gmres(lambda v: A @ v, lambda v: v, b, 1e-30, 50, k, record=True)
    assert it == k
    K = np.column_stack([np.linalg.matrix_power(A.toarray(), j) @ b for j in range(k)])
    Q, _ = np.linalg.qr(K)
    coef, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
    x_ls = Q @ coef
    np.testing.assert_allclose(x, x_ls, rtol=1e-8, atol=1e-10 * np.abs(x_ls).max())
    np.testing.assert_allclose(hist[-1]["x"], x, rtol=1e-12, atol=0)


def test_exact_preconditioner_one_step():
    A, b = _system()
    Ainv = direct.dense_inverse(A)
    x, it, rr, _ = gmres(lambda v: A @ v, lambda v: Ainv @ v, b, 1e-10, 20, 20)
    assert it == 1 and rr <= 1e-10


@pytest.mark.parametrize("restart", [3, 10, 60])
def test_restarted_converges_to_direct(restart):
    # no PML and a low frequency make -A symmetric positive definite, so every
    # restart length converges
    A, b = _system(8, omega=1.0, C=0.0)
    u = direct.solve(A, b)
    x, it, rr, hist = gmres(lambda v: A @ v, lambda v: v, b, 1e-11, restart, 3000)
    assert rr <= 1e-11
    assert np.linalg.norm(x - u) / np.linalg.norm(u) < 1e-7
    est = [h["relres_est"] for h in hist[:restart]]
    assert all(b_ <= a_ * (1 + 1e-12) for a_, b_ in zip(est, est[1:]))
