"""Pins of the oracle's point-block Jacobi preconditioner (right-preconditioned Bi-CGSTAB for Eq 21).

* the 3x3 diagonal blocks built from the sparse contrast operator and the Green's table equal the blocks
  read off the dense matrix A, at every cell, boundary and corner cells included, for an isotropic and an
  anisotropic (folded) background;
* the per-cell construction on a small window around each cell equals both;
* zero contrast gives D = I; a density-only contrast gives D(x) = (1 - w^2 drho(x) g0) I with g0 the
  closed-form self term of the Green's tensor;
* M^-1 inverts M cell by cell;
* right-preconditioned Bi-CGSTAB reaches the LU solution, and with M = I it is Bi-CGSTAB.
"""

import numpy as np
import pytest

from oracle import green, operator as op, precond, solve
from paper_2301_12836_amd import models

H = 10.0
W = 2 * np.pi * 15.0


def problem(shape, seed, rel=0.2, w=W, aniso=False):
    m = models.random_medium(shape, seed, rel=rel, h=H, aniso_background=aniso)
    return op.Problem(shape, H, m.C0, m.rho0, m.dc21, m.drho, w)


@pytest.mark.parametrize("shape,aniso", [((5, 4, 6), False), ((4, 6, 5), True), ((2, 3, 7), True)])
def test_sparse_blocks_equal_dense_blocks(shape, aniso):
    P = problem(shape, 11, aniso=aniso)
    Dd = precond.block_diagonal_dense(P)
    Ds = precond.block_diagonal(P)
    scale = np.abs(Dd).max()
    assert np.abs(Ds - Dd).max() <= 1e-13 * scale
    # the contrast really moves the blocks away from I, off-diagonal entries included
    off = Dd - np.eye(3)[None]
    assert np.abs(off[:, 0, 1]).max() > 1e-3 and np.abs(off[:, 2, 2]).max() > 1e-2


def test_window_blocks_equal_sparse_blocks():
    P = problem((7, 8, 9), 12, aniso=True)
    Ds = precond.block_diagonal(P)
    cells = np.array([(0, 0, 0), (6, 7, 8), (1, 4, 4), (3, 4, 4), (6, 0, 5), (2, 7, 1), (5, 1, 7)])
    Dw = precond.block_diagonal_at(P, cells)
    p = (cells[:, 2] * 8 + cells[:, 1]) * 7 + cells[:, 0]
    assert np.abs(Dw - Ds[p]).max() <= 1e-13 * np.abs(Ds).max()


def test_zero_contrast_gives_identity():
    m = models.random_medium((4, 5, 3), 3, rel=0.1, h=H)
    P = op.Problem(m.shape, H, m.C0, m.rho0, np.zeros_like(m.dc21), np.zeros_like(m.drho), W)
    assert np.abs(precond.block_diagonal(P) - np.eye(3)[None]).max() == 0.0


def test_density_contrast_closed_form():
    m = models.random_medium((5, 4, 4), 5, rel=0.1, h=H)
    drho = np.random.default_rng(7).normal(size=m.drho.shape) * 300.0
    P = op.Problem(m.shape, H, m.C0, m.rho0, np.zeros_like(m.dc21), drho, W)
    g0 = green.green_self_term(H, W, P.alpha, P.beta, P.rho0)
    want = (1.0 - W**2 * drho.reshape(-1)[:, None, None] * g0) * np.eye(3)[None]
    got = precond.block_diagonal(P)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_inverse_solves_every_block(rng):
    P = problem((4, 3, 5), 2, aniso=True)
    D = precond.block_diagonal(P)
    v = models.random_field(P.shape, 9)
    y = precond.apply_inverse(D, v)
    back = np.einsum('pij,jp->ip', D, y.reshape(3, -1)).reshape(v.shape)
    assert np.abs(back - v).max() <= 1e-13 * np.abs(v).max()


def test_right_preconditioned_bicgstab_reaches_lu_solution():
    P = problem((6, 5, 4), 13, rel=0.3, w=2 * np.pi * 30.0, aniso=True)
    b = P.rhs_moment(models.double_couple(30, 60, 90), (3, 2, 1))
    want = solve.solve_dense(P.dense_A(), b)
    D = precond.block_diagonal(P)
    x, hist, nmv = precond.bicgstab_right(P.apply_fft, lambda v: precond.apply_inverse(D, v), b, 1e-12)
    assert hist[-1] <= 1e-12
    assert np.linalg.norm((x - want).ravel()) <= 1e-10 * np.linalg.norm(want.ravel())
    # M = I: the textbook method, step for step
    x1, h1, n1 = precond.bicgstab_right(P.apply_fft, lambda v: v, b, 1e-12)
    x0, h0, n0 = solve.bicgstab(P.apply_fft, b, 1e-12)
    assert n1 == n0 and np.allclose(h1, h0, rtol=1e-9, atol=0)
    assert np.linalg.norm((x1 - x0).ravel()) <= 1e-12 * np.linalg.norm(x0.ravel())
