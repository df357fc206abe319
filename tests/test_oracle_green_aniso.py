"""Pins of the oracle's anisotropic background Green's tensor against facts fixed by the mathematics.

* an isotropic stiffness reduces it to the closed form of Eq 7 (Stokes' solution, itself pinned
  against Kelvin's solution, A.5 and the PDE in test_oracle_green.py), its self-term to the
  sphere-averaged isotropic self-term;
* for VTI, tilted (TTI) and orthorhombic media it solves the elastodynamic equation
  c_ijkl d_j d_l G_km + rho w^2 G_im = 0 away from the source, by independent finite differences,
  and its static part (w -> 0) the equation of elastostatics; a planted index error in the
  Christoffel contraction fails that check;
* symmetry (G = G^T), evenness (G(-x) = G(x)) and, for media with the three coordinate mirror
  planes, G_ij(s x) = s_i s_j G_ij(x);
* the anisotropic self-term equals a brute-force integral of G over the sphere of volume h^3;
* the quadrature has converged (doubling every node count changes nothing beyond rounding).
"""

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

from oracle import green, green_aniso as ga
from oracle.operator import iso_stiffness
from paper_2301_12836_amd import models

ALPHA, BETA, RHO = 3000.0, 1730.0, 2400.0
C_ISO = iso_stiffness(RHO * ALPHA**2, RHO * BETA**2)
C_VTI = models.vti_from_thomsen(3000.0, 1700.0, 0.1, 0.05, 0.08, RHO)
C_TTI = models.rotate_voigt(C_VTI, models.rot_z(45.0) @ models.rot_y(30.0))
C_ORTHO = models.ortho_background()[0]


@pytest.mark.parametrize("f", [1e-4, 15.0, 40.0])
def test_isotropic_stiffness_gives_the_closed_form(f):
    w = 2 * np.pi * f
    d = np.array([[10.0, 0.0, 0.0], [3.0, -4.0, 12.0], [80.0, 50.0, -120.0], [400.0, 300.0, 600.0],
                  [0.0, -250.0, 40.0]])
    g = ga.green_aniso(d, w, C_ISO, RHO)
    g0 = green.green_exact(d, w, ALPHA, BETA, RHO)
    for p in range(len(d)):
        assert np.abs(g[p] - g0[p]).max() <= 1e-12 * np.abs(g0[p]).max()


@pytest.mark.parametrize("f", [1e-4, 15.0, 40.0])
def test_isotropic_self_term(f):
    w = 2 * np.pi * f
    s = ga.green_aniso_self_term(8.0, w, C_ISO, RHO)
    s0 = green.green_self_term(8.0, w, ALPHA, BETA, RHO)
    assert np.abs(s - s0 * np.eye(3)).max() <= 1e-13 * abs(s0)


def elastic_residual(C, x0, w, step=0.5):
    """(c_ijkl d_j d_l G_km + rho w^2 G_im, scale) at x0 by 4th-order central differences."""
    c4 = ga.stiffness4(C)
    c1 = np.array([1.0 / 12, -2.0 / 3, 0.0, 2.0 / 3, -1.0 / 12])
    c2 = np.array([-1.0 / 12, 4.0 / 3, -5.0 / 2, 4.0 / 3, -1.0 / 12])
    off = np.arange(-2, 3)
    e = np.eye(3)
    pts, plan = [], []
    for j in range(3):
        for l in range(j, 3):
            for s in range(5):
                for t in range(5):
                    if j == l and s != 2:
                        continue
                    p = x0 + off[t] * step * e[l] + (off[s] * step * e[j] if j != l else 0.0)
                    plan.append((j, l, s, t))
                    pts.append(p)
    G = ga.green_aniso(np.array(pts + [x0]), w, C, RHO)
    D2 = np.zeros((3, 3, 3, 3), dtype=complex)       # [j, l, k, m] = d_j d_l G_km
    for (j, l, s, t), g in zip(plan, G[:-1]):
        wgt = c2[t] if j == l else c1[s] * c1[t]
        D2[j, l] += wgt * g / step**2
        if j != l:
            D2[l, j] += wgt * g / step**2
    elastic = np.einsum('ijkl,jlkm->im', c4, D2)
    inertia = RHO * w * w * G[-1]
    scale = max(np.abs(inertia).max(), np.abs(c4).max() * np.abs(D2).max())
    return elastic + inertia, scale


@pytest.mark.parametrize("name", ["vti", "tti", "ortho"])
@pytest.mark.parametrize("f", [12.0, 30.0])
def test_solves_the_elastodynamic_equation(name, f):
    C = {"vti": C_VTI, "tti": C_TTI, "ortho": C_ORTHO}[name]
    res, scale = elastic_residual(C, np.array([41.0, -23.0, 57.0]), 2 * np.pi * f)
    assert np.abs(res).max() < 1e-6 * scale


@pytest.mark.parametrize("name", ["vti", "ortho"])
def test_static_part_solves_elastostatics(name):
    C = {"vti": C_VTI, "ortho": C_ORTHO}[name]
    res, scale = elastic_residual(C, np.array([12.0, 30.0, -17.0]), 1e-9)
    assert np.abs(res).max() < 1e-6 * scale


def test_planted_index_error_fails_the_equation(monkeypatch):
    """Contracting the second index pair, c_ijkl n_k n_l, instead of c_ijkl n_j n_l must not pass the PDE check."""
    def wrong(C, n):
        return np.einsum('ijkl,...k,...l->...ij', ga.stiffness4(C), n, n)
    monkeypatch.setattr(ga, "christoffel", wrong)
    res, scale = elastic_residual(C_TTI, np.array([41.0, -23.0, 57.0]), 2 * np.pi * 12.0)
    assert np.abs(res).max() > 1e-3 * scale


def test_symmetries(rng):
    w = 2 * np.pi * 20.0
    d = rng.normal(size=(6, 3)) * 60.0
    for C in (C_VTI, C_TTI, C_ORTHO):
        g = ga.green_aniso(d, w, C, RHO)
        scale = np.abs(g).max()
        assert np.abs(g - np.swapaxes(g, -1, -2)).max() < 1e-14 * scale
        assert np.abs(g - ga.green_aniso(-d, w, C, RHO)).max() < 1e-12 * scale
    for C, mirrored in ((C_VTI, True), (C_ORTHO, True), (C_TTI, False)):
        g = ga.green_aniso(d, w, C, RHO)
        for sgn in (np.array([-1.0, 1.0, 1.0]), np.array([1.0, -1.0, 1.0]), np.array([1.0, 1.0, -1.0])):
            gm = ga.green_aniso(d * sgn, w, C, RHO)
            err = np.abs(gm - g * np.outer(sgn, sgn)).max() / np.abs(g).max()
            assert (err < 1e-12) if mirrored else (err > 1e-3)


@pytest.mark.parametrize("name", ["vti", "ortho", "tti"])
def test_self_term_is_the_ball_integral(name):
    """S = integral of G over the sphere of volume h^3: Gauss-Legendre in r and cos(theta), trapezoid in phi."""
    C = {"vti": C_VTI, "ortho": C_ORTHO, "tti": C_TTI}[name]
    h, w = 10.0, 2 * np.pi * 25.0
    a = green.SPHERE_RADIUS_FACTOR * h
    xr, wr = leggauss(8)
    xt, wt = leggauss(12)
    nphi = 16
    r = 0.5 * a * (xr + 1.0)
    wr = 0.5 * a * wr
    phi = 2 * np.pi * np.arange(nphi) / nphi
    R, CT, PH = np.meshgrid(r, xt, phi, indexing='ij')
    ST = np.sqrt(1 - CT**2)
    d = np.stack([R * ST * np.cos(PH), R * ST * np.sin(PH), R * CT], axis=-1)
    W = (wr[:, None, None] * wt[None, :, None] * (2 * np.pi / nphi)) * R**2
    G = ga.green_aniso(d.reshape(-1, 3), w, C, RHO).reshape(d.shape[:-1] + (3, 3))
    integral = np.einsum('abc,abcij->ij', W, G)
    s = ga.green_aniso_self_term(h, w, C, RHO)
    assert np.abs(integral - s).max() < 1e-7 * np.abs(s).max()


def test_quadrature_converged():
    """Doubling every node count changes nothing beyond rounding, also for a strongly anisotropic VTI
    medium (Thomsen epsilon 0.5, delta 0.2, gamma 0.4)."""
    w = 2 * np.pi * 35.0
    d = np.array([[300.0, 200.0, 500.0], [630.0, 0.0, 0.0], [10.0, 0.0, 0.0], [-40.0, 90.0, 7.0], [0.0, 0.0, 500.0]])
    c_strong = models.vti_from_thomsen(3000.0, 1400.0, 0.5, 0.2, 0.4, RHO)
    for C in (C_TTI, C_ORTHO, c_strong):
        g1 = ga.green_aniso(d, w, C, RHO)
        g2 = ga.green_aniso(d, w, C, RHO, scale=2.0)
        for p in range(len(d)):
            assert np.abs(g1[p] - g2[p]).max() < 1e-12 * np.abs(g2[p]).max()


@pytest.mark.slow
def test_uniform_vti_contrast_reproduces_the_vti_tensor():
    """Physics link between the two anisotropic formulations: a uniform VTI contrast over the isotropic
    background (the LS solve, damped frequency so the box edges fade) reproduces near the centre the
    field of the VTI medium's own Green's tensor, far closer than the isotropic incident field does."""
    from oracle import operator as op, solve
    n, h, rho0 = 12, 10.0, 2400.0
    shape = (n, n, n)
    c_iso = models.iso_C(3000.0, 1730.0, rho0)
    c_vti = models.vti_from_thomsen(3000.0, 1730.0, 0.1, 0.05, 0.08, rho0)
    w = 2 * np.pi * 6.0 * (1 + 0.6j)
    dc = np.broadcast_to(op.pack21(c_vti - c_iso)[:, None, None, None], (21, n, n, n)).copy()
    P = op.Problem(shape, h, c_iso, rho0, dc, np.zeros((n, n, n)), w)
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing='ij')
    c = (n - 1) / 2
    g = np.exp(-((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2) / (2 * 1.5**2))
    f = np.zeros((3, n, n, n), dtype=complex)
    f[0], f[2] = g, 0.5 * g
    b = op.convolve_fft(f, P.table())
    u, _, _ = solve.bicgstab(P.apply_fft, b, 1e-10, 400)
    Pa = op.Problem(shape, h, c_vti, rho0, np.zeros((21, n, n, n)), np.zeros((n, n, n)), w, mode='aniso')
    ref = op.convolve_fft(f, Pa.table())
    m = slice(4, 8)
    err = np.linalg.norm((u - ref)[:, m, m, m]) / np.linalg.norm(ref[:, m, m, m])
    base = np.linalg.norm((b - ref)[:, m, m, m]) / np.linalg.norm(ref[:, m, m, m])
    assert base > 0.06 and err < 0.025
