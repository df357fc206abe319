"""Pins of the oracle's discrete LS operator (Eq 8-21) against facts fixed by the mathematics and physics.

* the strain stencil is exact on linear displacement fields (Eq 17-18) and its
  adjoint satisfies summation by parts;
* three independent constructions of A u agree (dense matrix, per-cell direct
  sums with on-the-fly closed-form G, zero-padded FFT);
* zero contrast gives A = I and the incident field equals the central-difference
  moment stencil of the closed-form G, which converges at O(h^2) to the
  Aki-Richards form -M_jk dG_ij/dx_k built from the printed derivatives A.7-A.11;
* point-force and moment-tensor/strain reciprocity, mirror symmetry, the Born
  limit, and BiCGSTAB reaching the LU solution;
* physics: a uniform density or stiffness contrast reproduces the Green's
  tensor of the perturbed homogeneous medium.
"""

import numpy as np
import pytest

from oracle import green, operator as op, solve
from paper_2301_12836_amd import models

H = 10.0
W15 = 2 * np.pi * 15.0


def small_problem(shape, seed, rel=0.1, w=W15, aniso=False):
    m = models.random_medium(shape, seed, rel=rel, h=H, aniso_background=aniso)
    return op.Problem(shape, H, m.C0, m.rho0, m.dc21, m.drho, w)


def test_strain_exact_on_linear_fields(rng):
    shape = (5, 4, 6)
    g = rng.normal(size=(3, 3))            # du_c/dx_a = g[c, a]
    k, j, i = np.meshgrid(np.arange(6), np.arange(4), np.arange(5), indexing='ij')
    X = np.stack([i, j, k]).astype(float) * H
    u = np.einsum('ca,a...->c...', g, X) + rng.normal(size=(3, 1, 1, 1))
    eps = op.strain_apply(u, H)
    expect = [g[0, 0], g[1, 1], g[2, 2], g[1, 2] + g[2, 1], g[0, 2] + g[2, 0], g[0, 1] + g[1, 0]]
    for J in range(6):
        assert np.allclose(eps[J], expect[J], rtol=0, atol=1e-13)
    E = op.strain_operator(shape, H)
    assert np.allclose((E @ u.ravel()).reshape(eps.shape), eps, rtol=0, atol=1e-13)


def test_strain_adjoint_summation_by_parts(rng):
    for shape in [(2, 3, 4), (5, 5, 5), (7, 3, 2)]:
        n1, n2, n3 = shape
        u = rng.normal(size=(3, n3, n2, n1)) + 1j * rng.normal(size=(3, n3, n2, n1))
        tau = rng.normal(size=(6, n3, n2, n1)) + 1j * rng.normal(size=(6, n3, n2, n1))
        lhs = np.sum(tau * op.strain_apply(u, H))
        rhs = np.sum(op.strain_adjoint_apply(tau, H) * u)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)
        E = op.strain_operator(shape, H)
        assert np.allclose((E.T @ tau.ravel()).reshape(u.shape), op.strain_adjoint_apply(tau, H), atol=1e-14)


def test_contrast_sparse_equals_sliced(rng):
    P = small_problem((5, 4, 3), 3, aniso=True)
    u = models.random_field(P.shape, 4)
    a = (P.B() @ u.ravel()).reshape(u.shape)
    b = P.contrast(u)
    assert np.abs(a - b).max() < 1e-13 * np.abs(a).max()


def test_three_constructions_of_apply():
    P = small_problem((6, 5, 7), 11, aniso=True)
    u = models.random_field(P.shape, 5)
    dense = (P.dense_A() @ u.ravel()).reshape(u.shape)
    fft = P.apply_fft(u)
    brute = P.apply_bruteforce(u)
    cells = np.array([[0, 0, 0], [5, 4, 6], [2, 3, 1], [5, 0, 3]])
    direct = P.apply_bruteforce(u, cells)
    scale = np.abs(dense).max()
    assert np.abs(dense - fft).max() < 1e-13 * scale
    assert np.abs(dense - brute).max() < 1e-13 * scale
    assert np.abs(direct - dense[:, cells[:, 2], cells[:, 1], cells[:, 0]].T).max() < 1e-13 * scale


def test_zero_contrast_is_identity_and_rhs_is_moment_stencil():
    shape = (7, 6, 8)
    n1, n2, n3 = shape
    C0 = models.iso_C(3000.0, 1730.0, 2400.0)
    P = op.Problem(shape, H, C0, 2400.0, np.zeros((21, n3, n2, n1)), np.zeros((n3, n2, n1)), W15)
    assert np.array_equal(P.dense_A(), np.eye(3 * P.n))
    M = np.array([0.3, -1.1, 0.7, 0.25, -0.4, 0.9])          # Voigt 11,22,33,23,13,12
    Mt = np.array([[M[0], M[5], M[4]], [M[5], M[1], M[3]], [M[4], M[3], M[2]]])
    s = np.array([3, 2, 4])
    t0 = 0.013
    b = P.rhs_moment(M, tuple(s), t0)
    # direct: b_i(x) = e^{i w t0} sum_jk M_jk [G_ij(x-s-e_k h) - G_ij(x-s+e_k h)] / (2h), with the
    # self-term where an offset vanishes
    selfv = green.green_self_term(H, W15, P.alpha, P.beta, 2400.0) / H**3
    expect = np.zeros_like(b)
    for (i, j, k) in np.ndindex(n1, n2, n3):
        x = np.array([i, j, k])
        acc = np.zeros(3, dtype=complex)
        for kk in range(3):
            for sign in (+1, -1):
                off = (x - s - sign * np.eye(3, dtype=int)[kk]) * H
                if not off.any():
                    G = selfv * np.eye(3)
                else:
                    G = green.green_exact(off.astype(float), W15, P.alpha, P.beta, 2400.0)
                acc += sign * G @ Mt[:, kk] / (2 * H)
        expect[:, k, j, i] = acc * np.exp(1j * W15 * t0)
    assert np.abs(b - expect).max() < 1e-13 * np.abs(expect).max()


def test_rhs_converges_to_aki_richards_moment_field():
    """The discrete incident field tends to u0_i = -M_jk dG_ij/dx_k (x - s) (Eq 15-16, A.7-A.11) at O(h^2)."""
    C0 = models.iso_C(3000.0, 1730.0, 2400.0)
    M = np.array([0.3, -1.1, 0.7, 0.25, -0.4, 0.9])
    Mt = np.array([[M[0], M[5], M[4]], [M[5], M[1], M[3]], [M[4], M[3], M[2]]])
    w = 2 * np.pi * 10.0
    errs = []
    for h in (8.0, 4.0, 2.0):
        n = int(round(48.0 / h)) + 1
        s = np.array([n // 4, n // 4, n // 4])
        P = op.Problem((n, n, n), h, C0, 2400.0, np.zeros((21, n, n, n)), np.zeros((n, n, n)), w, mode='paper_sum')
        f = P.moment_source(M, tuple(s))
        cell = s + np.array([int(24 / h), int(16 / h), int(32 / h)])   # fixed physical offset (24, 16, 32) m
        b = op.convolve_at(f, P.shape, h, w, P.alpha, P.beta, 2400.0, cell[None], mode='paper_sum')[0]
        dG = green.green_paper_sum_grad(np.array([24.0, 16.0, 32.0]), w, P.alpha, P.beta, 2400.0)
        exact = -np.einsum('jk,ijk->i', Mt, dG)
        errs.append(np.abs(b - exact).max() / np.abs(exact).max())
    assert errs[0] < 0.1
    assert 3.3 < errs[0] / errs[1] < 4.7 and 3.3 < errs[1] / errs[2] < 4.7


def test_point_force_and_moment_strain_reciprocity():
    P = small_problem((5, 4, 6), 21, rel=0.15, aniso=True)
    A = P.dense_A()
    r, s = (1, 2, 4), (3, 1, 2)
    sol = {}
    for cell in (r, s):
        for c in range(3):
            F = np.eye(3)[c]
            sol[cell, c] = solve.solve_dense(A, P.rhs_force(F, cell))
    for i in range(3):
        for j in range(3):
            a = sol[s, j][i, r[2], r[1], r[0]]
            b = sol[r, i][j, s[2], s[1], s[0]]
            assert abs(a - b) < 1e-11 * max(abs(a), abs(b))
    # u_i(r; M at s) = sum_J M_J eps_J(s) of the field of a unit force e_i at r
    M = np.array([0.5, -0.2, 0.9, 0.1, 0.6, -0.3])
    u = solve.solve_dense(A, P.rhs_moment(M, s))
    for i in range(3):
        eps = op.strain_apply(sol[r, i], P.h)[:, s[2], s[1], s[0]]
        lhs = u[i, r[2], r[1], r[0]]
        rhs = np.dot(M, eps)
        assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_mirror_symmetry_of_centred_explosion():
    m = models.config1(n=9)
    P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, W15)
    u = solve.solve_dense(P.dense_A(), P.rhs_moment(models.EXPLOSION, (4, 4, 4)))
    # reflect x: u_x odd, u_y and u_z even
    assert np.allclose(u[0], -u[0][:, :, ::-1], atol=1e-13 * np.abs(u).max())
    assert np.allclose(u[1], u[1][:, :, ::-1], atol=1e-13 * np.abs(u).max())
    # cubic symmetry: swapping x and y swaps u_x and u_y
    assert np.allclose(u[0], np.swapaxes(u[1], 1, 2), atol=1e-13 * np.abs(u).max())


def test_born_limit_slope_two():
    P1 = small_problem((5, 5, 5), 7, rel=0.1)
    b = P1.rhs_moment(models.double_couple(30, 60, 90), (2, 2, 2))
    errs = []
    for scale in (1e-1, 1e-2, 1e-3):
        P = op.Problem(P1.shape, H, models.iso_C(3000.0, 1730.0, 2400.0), 2400.0, scale * P1.dc21,
                       scale * P1.drho, W15)
        u = solve.solve_dense(P.dense_A(), b)
        born = b + (b - P.apply_fft(b))   # b + K b with K = I - A
        errs.append(np.linalg.norm(u - born))
    slopes = np.log10(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 2.0) < 0.1)


def test_density_point_scatterer():
    """Single-cell density contrast: (I - A) u = w^2 drho h^3 G(x - p) u(p) (Eq 8's density term)."""
    shape = (5, 6, 4)
    n1, n2, n3 = shape
    p = (2, 3, 1)
    drho = np.zeros((n3, n2, n1))
    drho[p[2], p[1], p[0]] = 37.0
    C0 = models.iso_C(3000.0, 1730.0, 2400.0)
    P = op.Problem(shape, H, C0, 2400.0, np.zeros((21, n3, n2, n1)), drho, W15)
    u = models.random_field(shape, 8)
    cells = np.array([(0, 0, 0), (4, 5, 3), (2, 3, 1)])
    Ku = op.convolve_at(P.contrast(u), shape, H, W15, P.alpha, P.beta, 2400.0, cells)
    assert np.allclose(Ku.T, (u - P.apply_bruteforce(u))[:, cells[:, 2], cells[:, 1], cells[:, 0]],
                       rtol=1e-9, atol=0)
    up = u[:, p[2], p[1], p[0]]
    for t, (i, j, k) in enumerate(cells):
        off = np.array([i - p[0], j - p[1], k - p[2]], dtype=float) * H
        if off.any():
            G = green.green_exact(off, W15, P.alpha, P.beta, 2400.0) * H**3
        else:
            G = green.green_self_term(H, W15, P.alpha, P.beta, 2400.0) * np.eye(3)
        expect = W15**2 * 37.0 * G @ up
        assert np.allclose(Ku[t], expect, rtol=1e-12, atol=0)


def _uniform_contrast_error(dc66, drho_val, alpha1, beta1, rho1):
    n = 20
    shape = (n, n, n)
    rho0 = 2400.0
    C0 = models.iso_C(3000.0, 1730.0, rho0)
    w = 2 * np.pi * 6.0 * (1 + 0.6j)          # damped frequency: boundary reflections decay
    dc = np.broadcast_to(op.pack21(dc66)[:, None, None, None], (21, n, n, n)).copy()
    P = op.Problem(shape, H, C0, rho0, dc, np.full((n, n, n), drho_val), w)
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing='ij')
    c = (n - 1) / 2
    g = np.exp(-((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2) / (2 * 1.5**2))
    f = np.zeros((3, n, n, n), dtype=complex)
    f[0], f[2] = g, 0.5 * g
    b = op.convolve_fft(f, P.table())
    u, _, _ = solve.bicgstab(P.apply_fft, b, 1e-10, 400)
    ref = op.convolve_fft(f, op.green_table(shape, H, w, alpha1, beta1, rho1))
    m = slice(6, 14)
    err = np.linalg.norm((u - ref)[:, m, m, m]) / np.linalg.norm(ref[:, m, m, m])
    born0 = np.linalg.norm((b - ref)[:, m, m, m]) / np.linalg.norm(ref[:, m, m, m])
    return err, born0


@pytest.mark.slow
def test_uniform_density_contrast_gives_perturbed_green_tensor():
    rho0, eps = 2400.0, 0.2
    err, base = _uniform_contrast_error(np.zeros((6, 6)), eps * rho0, 3000.0 / np.sqrt(1 + eps),
                                        1730.0 / np.sqrt(1 + eps), rho0 * (1 + eps))
    assert base > 0.05 and err < 0.02


@pytest.mark.slow
def test_uniform_stiffness_contrast_gives_perturbed_green_tensor():
    rho0 = 2400.0
    lam0, mu0 = rho0 * (3000.0**2 - 2 * 1730.0**2), rho0 * 1730.0**2
    lam1, mu1 = 1.1 * lam0, 1.25 * mu0
    C1 = models.iso_C(np.sqrt((lam1 + 2 * mu1) / rho0), np.sqrt(mu1 / rho0), rho0)
    dc66 = C1 - models.iso_C(3000.0, 1730.0, rho0)
    err, base = _uniform_contrast_error(dc66, 0.0, np.sqrt((lam1 + 2 * mu1) / rho0), np.sqrt(mu1 / rho0), rho0)
    assert base > 0.1 and err < 0.04


def test_vti_background_folds_to_thomsen_reference():
    m = models.config2(n=6)
    alpha, beta, c_iso = op.iso_reference(m.C0, m.rho0)
    assert abs(alpha - 3000.0) < 1e-9 and abs(beta - 1700.0) < 1e-9
    P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, W15)
    total = op.unpack21(P.dc21)[:, :, 0, 0, 0]
    assert np.allclose(total + c_iso, m.C0 + op.unpack21(m.dc21)[:, :, 0, 0, 0], rtol=1e-14, atol=0)


def test_bicgstab_reaches_lu_solution():
    m = models.config1(n=8)
    P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, W15)
    b = P.rhs_moment(models.EXPLOSION, (2, 4, 4))
    x_lu = solve.solve_dense(P.dense_A(), b)
    x, hist, nmv = solve.bicgstab(P.apply_fft, b, 1e-12)
    assert hist[-1] <= 1e-12
    assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) < 1e-10
    assert solve.relative_residual(P.apply_fft, x, b) < 1e-11


def test_taper_weights_geometry():
    """Absorbing-layer weights (Eq 23-25): 1 outside the layer; on the axis through the centre of a face the
    ray meets that face at right angles, so l is the distance from the cell centre to the face; the
    weights share the grid's mirror symmetries and grow along a ray away from the boundary."""
    shape, d = (14, 12, 10), 3
    w = op.taper_weights(shape, d)
    assert w.shape == (10, 12, 14)
    assert np.all(w[d:10 - d, d:12 - d, d:14 - d] == 1.0)
    assert np.all((w > 0) & (w <= 1))
    # mirror symmetries of the box
    assert np.allclose(w, w[::-1]) and np.allclose(w, w[:, ::-1]) and np.allclose(w, w[:, :, ::-1])
    # on an odd cube the centre is a cell, so the axis lines through it are face-normal rays
    w2 = op.taper_weights((9, 9, 9), 2)
    for i, dist in [(0, 0.5), (1, 1.5), (8, 0.5), (7, 1.5)]:
        assert np.isclose(w2[4, 4, i], 1.0 - np.exp(-dist ** 2 / 9.0))
        assert np.isclose(w2[i, 4, 4], 1.0 - np.exp(-dist ** 2 / 9.0))
    # along the diagonal ray from the centre the weight increases inwards
    diag = [w2[k, k, k] for k in range(2)]
    assert diag[0] < diag[1]
    # the corner cell's ray leaves through the corner: l = sqrt(3) / 2
    assert np.isclose(w2[0, 0, 0], 1.0 - np.exp(-0.75 / 9.0))
    assert np.all(op.taper_weights(shape, 0) == 1.0)


def test_bicgstab_l_with_one_step_is_bicgstab():
    """BiCGSTAB(1) and the textbook Bi-CGSTAB are the same method: equal residual histories."""
    P = small_problem((6, 5, 7), 31, rel=0.3)
    b = P.rhs_moment(models.EXPLOSION, (2, 2, 3))
    _, h1, n1 = solve.bicgstab(P.apply_fft, b, 1e-11)
    _, hl, nl = solve.bicgstab_l(P.apply_fft, b, 1e-11, 1)
    assert len(h1) == len(hl) and nl == n1
    # rounding differences grow along the iteration; the first dozen steps agree to 1e-9
    assert np.allclose(hl[:12], h1[:12], rtol=1e-9, atol=0)


@pytest.mark.parametrize("ell", [2, 3, 4])
def test_bicgstab_l_reaches_lu_solution(ell):
    P = small_problem((6, 5, 7), 31, rel=0.3)
    b = P.rhs_moment(models.EXPLOSION, (2, 2, 3))
    x_lu = solve.solve_dense(P.dense_A(), b)
    x, hist, nmv = solve.bicgstab_l(P.apply_fft, b, 1e-12, ell)
    assert hist[-1] <= 1e-12
    # the recursively updated residual is the true one
    assert abs(solve.relative_residual(P.apply_fft, x, b) - hist[-1]) < 1e-12
    assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) < 1e-10


def test_model1_vti_folds_to_the_printed_isotropic_background():
    from golden_fixtures import load_model1
    """The paper's worked example: its VTI stiffness splits into the isotropic background it prints (c11 = 26.5,
    c44 = 10.4 GPa) plus a contrast; the oracle's reference-medium rule reproduces that background."""
    C, rho, c11, c44 = load_model1()
    alpha, beta, c_iso = op.iso_reference(C, rho)
    assert abs(c_iso[0, 0] - c11) < 1e-6 and abs(c_iso[3, 3] - c44) < 1e-6
    assert abs(alpha - np.sqrt(c11 / rho)) < 1e-9 and abs(beta - np.sqrt(c44 / rho)) < 1e-9
    total = op.unpack21(op.total_contrast21(C, rho, np.zeros((21, 1, 1, 1))))[:, :, 0, 0, 0]
    assert np.allclose(total + c_iso, C, rtol=0, atol=1e-3)
