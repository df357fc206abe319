"""Solvers for A u = b (oracle, test infrastructure only).

* ``solve_dense``: the exact discrete solution by LU (LAPACK through scipy).
  BiCGSTAB, on convergence, reaches this unique solution, so it is the plain
  definition of the result of the iterative solve (Eq 21-22).
* ``bicgstab``: van der Vorst's Bi-CGSTAB (the solver named for Eq 21), textbook
  form, unpreconditioned, x0 = 0 unless given, shadow residual r^ = r0, Hermitian
  inner products, relative residual e = ||b - A x|| / ||b|| of Eq 22 as the
  stopping rule.
"""

import numpy as np
import scipy.linalg as sla


def solve_dense(A, b):
    shape = b.shape
    return sla.solve(A, b.reshape(-1)).reshape(shape)


def relative_residual(apply_A, x, b):
    """Eq 22."""
    return np.linalg.norm((b - apply_A(x)).ravel()) / np.linalg.norm(b.ravel())


def bicgstab(apply_A, b, tol, maxit=2000, x0=None):
    """Returns (x, history, n_matvec); history holds e after every half and full step."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    nmv = 0 if x0 is None else 1
    bnorm = np.linalg.norm(b.ravel())
    if bnorm == 0.0:
        return np.zeros_like(b), [0.0], nmv
    rhat = r.copy()
    rho_old = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    hist = [np.linalg.norm(r.ravel()) / bnorm]
    for _ in range(maxit):
        rho = np.vdot(rhat, r)
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = apply_A(p)
        nmv += 1
        alpha = rho / np.vdot(rhat, v)
        s = r - alpha * v
        e = np.linalg.norm(s.ravel()) / bnorm
        if e <= tol:
            x = x + alpha * p
            hist.append(e)
            break
        t = apply_A(s)
        nmv += 1
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho_old = rho
        e = np.linalg.norm(r.ravel()) / bnorm
        hist.append(e)
        if e <= tol:
            break
    return x, hist, nmv
