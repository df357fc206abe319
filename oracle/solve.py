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


def bicgstab_l(apply_A, b, tol, ell, maxit=2000, x0=None):
    """BiCGSTAB(l) of Sleijpen and Fokkema (1993): l Bi-CG steps, then a minimal-residual polynomial of
    degree l over the l + 1 residuals the steps produced (modified Gram-Schmidt).  l = 1 is Bi-CGSTAB.

    Returns (x, history, n_matvec); history holds e after every Bi-CG step, the last step of each
    cycle after its minimal-residual update.  ``maxit`` bounds the number of Bi-CG steps."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = np.linalg.norm(b.ravel())
    nmv = 0 if x0 is None else 1
    if bnorm == 0.0:
        return np.zeros_like(b), [0.0], nmv
    r = [b - apply_A(x) if x0 is not None else b.copy()] + [None] * ell
    u = [np.zeros_like(b)] + [None] * ell
    rhat = r[0].copy()
    rho0 = alpha = omega = 1.0 + 0j
    alpha = 0.0 + 0j
    hist = [np.linalg.norm(r[0].ravel()) / bnorm]
    steps = 0
    while hist[-1] > tol and steps < maxit:
        rho0 = -omega * rho0
        for j in range(ell):                                # Bi-CG part
            rho1 = np.vdot(rhat, r[j])
            beta = alpha * rho1 / rho0
            rho0 = rho1
            for i in range(j + 1):
                u[i] = r[i] - beta * u[i]
            u[j + 1] = apply_A(u[j])
            alpha = rho0 / np.vdot(rhat, u[j + 1])
            for i in range(j + 1):
                r[i] = r[i] - alpha * u[i + 1]
            x = x + alpha * u[0]
            steps += 1
            e = np.linalg.norm(r[0].ravel()) / bnorm
            if e <= tol:                                    # converged inside the Bi-CG part
                hist.append(e)
                return x, hist, nmv + 2 * steps - 1
            r[j + 1] = apply_A(r[j])
            if j < ell - 1:
                hist.append(e)
        tau = np.zeros((ell + 1, ell + 1), dtype=complex)   # minimal-residual part
        sigma = np.zeros(ell + 1)
        gp = np.zeros(ell + 1, dtype=complex)
        for j in range(1, ell + 1):
            for i in range(1, j):
                tau[i, j] = np.vdot(r[i], r[j]) / sigma[i]
                r[j] = r[j] - tau[i, j] * r[i]
            sigma[j] = np.vdot(r[j], r[j]).real
            gp[j] = np.vdot(r[j], r[0]) / sigma[j]
        g = np.zeros(ell + 1, dtype=complex)
        g[ell] = gp[ell]
        omega = g[ell]
        for j in range(ell - 1, 0, -1):
            g[j] = gp[j] - sum(tau[j, i] * g[i] for i in range(j + 1, ell + 1))
        g2 = np.zeros(ell + 1, dtype=complex)
        for j in range(1, ell):
            g2[j] = g[j + 1] + sum(tau[j, i] * g[i + 1] for i in range(j + 1, ell))
        x = x + g[1] * r[0]
        r[0] = r[0] - gp[ell] * r[ell]
        u[0] = u[0] - g[ell] * u[ell]
        for j in range(1, ell):
            u[0] = u[0] - g[j] * u[j]
            x = x + g2[j] * r[j]
            r[0] = r[0] - gp[j] * r[j]
        hist.append(np.linalg.norm(r[0].ravel()) / bnorm)
    return x, hist, nmv + 2 * steps
