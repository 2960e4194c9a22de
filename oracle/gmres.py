"""Restarted GMRES with right preconditioning.  Parity pinned (Krylov
least-squares minimiser computed independently with numpy QR/lstsq, and
convergence to the direct solution; tests/test_oracle_gmres.py).

The paper uses "standard GMRES" with a relative-residual stop and a restart
length (Section 3.2) and does not state the side of preconditioning, the
initial guess or the orthogonalization.  This is the textbook method (Saad and
Schultz, 1986): x0 = 0, modified Gram-Schmidt Arnoldi on A M^-1, the small
least-squares problem min || beta e1 - Hbar y || solved at each step, inner stop
when its residual norm relative to ||b|| is <= tol, x = x0 + M^-1 (V y) at the
end of a cycle, and a restart while the true relative residual
||b - A x|| / ||b|| exceeds tol.  ``iters`` counts Arnoldi steps
(= preconditioner applies inside the cycles).
"""
import numpy as np


def gmres(A_mv, M_apply, b, tol, restart, maxit, record=False):
    """Returns (x, iters, true_relres, history); history holds the estimated
    relative residual after every Arnoldi step (and the iterate, if record)."""
    b = np.asarray(b, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b)
    iters = 0
    history = []
    if bnorm == 0.0:
        return x, 0, 0.0, history
    while True:
        r = b - A_mv(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol or iters >= maxit:
            return x, iters, beta / bnorm, history
        V = [r / beta]
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        y = None
        for j in range(restart):
            w = A_mv(M_apply(V[j]))
            for i in range(j + 1):                      # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            iters += 1
            e1 = np.zeros(j + 2, dtype=np.complex128)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[: j + 2, : j + 1], e1, rcond=None)
            est = np.linalg.norm(e1 - H[: j + 2, : j + 1] @ y) / bnorm
            entry = {"iter": iters, "relres_est": est}
            if record:
                entry["x"] = x + M_apply(np.column_stack(V[: j + 1]) @ y)
            history.append(entry)
            if est <= tol or iters >= maxit or H[j + 1, j] == 0.0:
                break
            V.append(w / H[j + 1, j])
        x = x + M_apply(np.column_stack(V[: len(y)]) @ y)
