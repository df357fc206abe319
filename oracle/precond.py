"""Point-block Jacobi preconditioning of the LS system (oracle, test infrastructure only).

The paper's concluding remarks name preconditioning as the way to speed up the iterative solve of Eq 21
without fixing a preconditioner.  The one restated here is the textbook point-block Jacobi
preconditioner:

    M = blockdiag_x D(x),   D(x) = [A]_(x,x), the 3x3 block of A = I - Gconv B (Eq 19-21) that couples the
                            three displacement components at cell x with themselves,

applied on the right (Barrett et al. 1994, preconditioned Bi-CGSTAB): Bi-CGSTAB runs on A M^-1 y = b and
returns x = M^-1 y, the solution of the unpreconditioned system.

* ``block_diagonal_dense``: D read off the dense matrix of ``operator.Problem.dense_A`` (the plain
  definition; tiny grids only).
* ``block_diagonal``: the same blocks without forming A, from the sparse contrast operator B and the
  Green's table:  D(x)_ic = delta_ic - sum_{x'} sum_j h^3 G_ij(x - x') B[(j, x'), (c, x)].  Column (c, x)
  of B reaches only cells within two cells of x (a strain stencil followed by its adjoint), so only the
  offsets in [-2, 2]^3 of the table enter.
* ``block_diagonal_at``: the same sum at listed cells only, with column (c, x) of B taken by applying the
  contrast operator to a unit vector on the cells within three of x (any size of grid).
* ``apply_inverse``: M^-1 v, one 3x3 solve per cell.
* ``bicgstab_right``: right-preconditioned Bi-CGSTAB.
"""

import numpy as np
import scipy.sparse as sp

from . import operator as op


def local_table(P):
    """h^3 G at the offsets [-2, 2]^3: T[3, 3, 5, 5, 5], offset (dx, dy, dz) at [..., dz+2, dy+2, dx+2]."""
    return op.green_table((3, 3, 3), P.h, P.omega, P.alpha, P.beta, P.rho0, P.mode, P.C0)


def block_diagonal_dense(P):
    """D [n, 3, 3] from the dense A (unknown c of cell p at row c n + p)."""
    A = P.dense_A()
    n = P.n
    idx = np.arange(n)
    D = np.empty((n, 3, 3), dtype=complex)
    for i in range(3):
        for c in range(3):
            D[:, i, c] = A[i * n + idx, c * n + idx]
    return D


def block_diagonal(P):
    """D [n, 3, 3] from the sparse B and the Green's table."""
    n = P.n
    T = local_table(P)
    B = sp.csc_matrix(P.B())
    col = np.repeat(np.arange(3 * n), np.diff(B.indptr))
    c, p = np.divmod(col, n)                 # B column (c, x = p)
    j, q = np.divmod(B.indices, n)           # B row (j, x' = q)
    xyz = op.cell_coords(P.shape)
    off = xyz[p] - xyz[q]                    # x - x'
    assert off.size == 0 or np.abs(off).max() <= 2
    g = T[:, j, off[:, 2] + 2, off[:, 1] + 2, off[:, 0] + 2]     # [3, nnz]
    D = np.zeros((n, 3, 3), dtype=complex)
    flat = D.reshape(-1)
    for i in range(3):
        np.add.at(flat, p * 9 + i * 3 + c, -g[i] * B.data)
    D[:, [0, 1, 2], [0, 1, 2]] += 1.0
    return D


def block_diagonal_at(P, cells):
    """D [m, 3, 3] at the listed cells ([m, 3] as (x, y, z))."""
    T = local_table(P)
    n1, n2, n3 = P.shape
    out = np.empty((len(cells), 3, 3), dtype=complex)
    for t, (i, j, k) in enumerate(np.asarray(cells)):
        lo = [max(v - 3, 0) for v in (i, j, k)]
        hi = [min(v + 4, m) for v, m in zip((i, j, k), (n1, n2, n3))]
        win = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
        dc = P.dc21[(slice(None),) + win]
        dr = P.drho[win]
        zz, yy, xx = np.meshgrid(np.arange(lo[2], hi[2]), np.arange(lo[1], hi[1]), np.arange(lo[0], hi[0]),
                                 indexing='ij')
        ox, oy, oz = i - xx, j - yy, k - zz
        near = (np.abs(ox) <= 2) & (np.abs(oy) <= 2) & (np.abs(oz) <= 2)
        g = T[:, :, oz[near] + 2, oy[near] + 2, ox[near] + 2]     # [3, 3, m]
        for c in range(3):
            u = np.zeros((3,) + dr.shape, dtype=complex)
            u[c, k - lo[2], j - lo[1], i - lo[0]] = 1.0
            f = op.contrast_apply(u, P.h, dc, dr, P.omega)
            assert not np.any(f[:, ~near])
            out[t, :, c] = -np.einsum('ijm,jm->i', g, f[:, near])
            out[t, c, c] += 1.0
    return out


def apply_inverse(D, v):
    """M^-1 v for v [3, N3, N2, N1]: the 3x3 system D(x) y(x) = v(x) at every cell."""
    y = np.linalg.solve(D, v.reshape(3, -1).T[:, :, None])[:, :, 0]
    return y.T.reshape(v.shape)


def bicgstab_right(apply_A, apply_Minv, b, tol, maxit=2000):
    """Bi-CGSTAB on A M^-1 y = b, x = M^-1 y: x0 = 0, shadow residual r0, Hermitian products, relative
    residual of Eq 22 checked after each half step.  Returns (x, history, n_matvec)."""
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = np.linalg.norm(b.ravel())
    if bnorm == 0.0:
        return x, [0.0], 0
    rhat = r.copy()
    rho_old = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    hist = [1.0]
    nmv = 0
    for _ in range(maxit):
        rho = np.vdot(rhat, r)
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        ph = apply_Minv(p)
        v = apply_A(ph)
        nmv += 1
        alpha = rho / np.vdot(rhat, v)
        s = r - alpha * v
        e = np.linalg.norm(s.ravel()) / bnorm
        if e <= tol:
            x = x + alpha * ph
            hist.append(e)
            break
        sh = apply_Minv(s)
        t = apply_A(sh)
        nmv += 1
        omega = np.vdot(t, s) / np.vdot(t, t)
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        rho_old = rho
        e = np.linalg.norm(r.ravel()) / bnorm
        hist.append(e)
        if e <= tol:
            break
    return x, hist, nmv
