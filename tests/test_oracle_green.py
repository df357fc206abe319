"""Pins of the oracle's Green's tensor (Eq 7, Appendix A) against facts fixed by the mathematics.

Each test checks the oracle against something other than itself: Kelvin's static
solution and its first-order frequency correction, the far-field tensor A.5, the
defining PDE (Eq 7) evaluated by independent finite differences, a numerical
quadrature of the self-term, and finite differences of A.4 + A.5 for the printed
derivative formulas A.7/A.9/A.11.
"""

import numpy as np
import pytest
from scipy.special import roots_legendre

from oracle import green

ALPHA, BETA, RHO = 3000.0, 1730.0, 2400.0


def kelvin_static(d, alpha, beta, rho):
    """Kelvin's solution for a unit point force in an isotropic solid (textbook closed form)."""
    r = np.linalg.norm(d)
    g = d / r
    return ((1.0 + beta**2 / alpha**2) * np.eye(3) + (1.0 - beta**2 / alpha**2) * np.outer(g, g)) \
        / (8.0 * np.pi * rho * beta**2 * r)


def test_symmetric_and_even(rng):
    d = rng.normal(size=(50, 3)) * 40.0
    for fn in (green.green_exact, green.green_paper_sum):
        G = fn(d, 2 * np.pi * 17.0, ALPHA, BETA, RHO)
        assert np.allclose(G, np.swapaxes(G, -1, -2), rtol=0, atol=1e-15 * np.abs(G).max())
        assert np.allclose(G, fn(-d, 2 * np.pi * 17.0, ALPHA, BETA, RHO), rtol=1e-14, atol=0)


@pytest.mark.parametrize("d", [np.array([3.0, -4.0, 12.0]), np.array([0.0, 0.0, 7.5]), np.array([20.0, 1.0, 0.5])])
def test_static_limit_and_first_order_term(d):
    """w -> 0: G -> Kelvin + i w (2/b^3 + 1/a^3)/(12 pi rho) I + O(w^2 r)."""
    K = kelvin_static(d, ALPHA, BETA, RHO)
    first = (2.0 / BETA**3 + 1.0 / ALPHA**3) / (12.0 * np.pi * RHO)
    for w in (1e-2, 1e-1, 1.0):
        G = green.green_exact(d, w, ALPHA, BETA, RHO)
        resid = G - K - 1j * w * first * np.eye(3)
        # second-order remainder: |G''| ~ r / (rho b^4) up to O(1) factors
        bound = 0.2 * w**2 * np.linalg.norm(d) / (RHO * BETA**4)
        assert np.abs(resid).max() < bound + 1e-15 * np.abs(K).max()
    # the paper's near-field tensor A.4 plus A.5 also reduces to Kelvin at w = 0 (same static limit)
    Gs = green.green_paper_sum(d, 1e-9, ALPHA, BETA, RHO)
    assert np.allclose(Gs, K, rtol=1e-9, atol=0)


def test_far_field_limit_is_A5():
    """k r >> 1: the exact tensor approaches the far-field tensor A.5 with an O(1/(k r)) remainder."""
    w = 2 * np.pi * 15.0
    for r in (1e4, 1e5, 1e6):
        d = r * np.array([0.48, -0.6, 0.64])
        g = d / r
        a5 = (np.exp(1j * w * r / ALPHA) * np.outer(g, g) / (4 * np.pi * RHO * r * ALPHA**2)
              + np.exp(1j * w * r / BETA) * (np.eye(3) - np.outer(g, g)) / (4 * np.pi * RHO * r * BETA**2))
        G = green.green_exact(d, w, ALPHA, BETA, RHO)
        rel = np.abs(G - a5).max() / np.abs(a5).max()
        assert rel < 3.0 / (w * r / BETA)


def navier_residual(fn, x0, w, step):
    """(l+m) grad div G + m lap G + rho w^2 G at x0, by 4th-order central differences (columns = force dirs)."""
    lam = RHO * (ALPHA**2 - 2 * BETA**2)
    mu = RHO * BETA**2
    c4 = np.array([1.0 / 12, -2.0 / 3, 0.0, 2.0 / 3, -1.0 / 12])
    c4_2 = np.array([-1.0 / 12, 4.0 / 3, -5.0 / 2, 4.0 / 3, -1.0 / 12])
    offs = np.arange(-2, 3)

    def G(x):
        return fn(x, w, ALPHA, BETA, RHO)

    e = np.eye(3)
    lap = np.zeros((3, 3), dtype=complex)
    for a in range(3):
        lap += sum(c4_2[t] * G(x0 + offs[t] * step * e[a]) for t in range(5)) / step**2
    # grad div: d_i d_k G_kn
    hess = np.zeros((3, 3, 3, 3), dtype=complex)   # [i, k] second derivative of G (component k, n)
    for i in range(3):
        for k in range(3):
            acc = 0
            for s in range(5):
                for t in range(5):
                    acc = acc + c4[s] * c4[t] * G(x0 + offs[s] * step * e[i] + offs[t] * step * e[k])
            hess[i, k] = acc / step**2
    graddiv = np.einsum('ikkn->in', hess)
    return (lam + mu) * graddiv + mu * lap + RHO * w**2 * G(x0)


def test_exact_mode_solves_eq7_and_paper_sum_does_not():
    w = 2 * np.pi * 12.0
    x0 = np.array([41.0, -23.0, 57.0])
    res = navier_residual(green.green_exact, x0, w, 0.5)
    scale = RHO * w**2 * np.abs(green.green_exact(x0, w, ALPHA, BETA, RHO)).max()
    assert np.abs(res).max() / scale < 1e-6
    res_sum = navier_residual(green.green_paper_sum, x0, w, 0.5)
    assert np.abs(res_sum).max() / scale > 1e-2   # A.4 + A.5 is not a solution of Eq 7 (near-field reading)


@pytest.mark.parametrize("f", [0.5, 15.0, 40.0])
def test_self_term_equals_sphere_quadrature(f):
    """h^3 G(0) = integral of G over the sphere of volume h^3 (Gauss-Legendre in r and cos(theta), trapezoid in phi)."""
    h = 8.0
    w = 2 * np.pi * f
    a = green.SPHERE_RADIUS_FACTOR * h
    xr, wr = roots_legendre(24)
    xt, wt = roots_legendre(16)
    nphi = 16
    r = 0.5 * a * (xr + 1.0)
    wr = 0.5 * a * wr
    phi = 2 * np.pi * np.arange(nphi) / nphi
    R, CT, PH = np.meshgrid(r, xt, phi, indexing='ij')
    ST = np.sqrt(1 - CT**2)
    d = np.stack([R * ST * np.cos(PH), R * ST * np.sin(PH), R * CT], axis=-1)
    W = (wr[:, None, None] * wt[None, :, None] * (2 * np.pi / nphi)) * R**2
    G = green.green_exact(d.reshape(-1, 3), w, ALPHA, BETA, RHO).reshape(d.shape[:-1] + (3, 3))
    integral = np.einsum('abc,abcij->ij', W, G)
    s = green.green_self_term(h, w, ALPHA, BETA, RHO)
    assert np.allclose(integral, s * np.eye(3), rtol=0, atol=1e-11 * abs(s))


def test_appendix_derivatives_match_finite_differences(rng):
    """A.7 + A.9 + A.11 (as printed, E_kl = delta_kl - 3 x_k x_l / r^2) equal d/dx_i of A.4 + A.5."""
    w = 2 * np.pi * 22.0
    for _ in range(5):
        d0 = rng.normal(size=3) * 30.0
        dG = green.green_paper_sum_grad(d0, w, ALPHA, BETA, RHO)
        step = 1e-3
        fd = np.zeros((3, 3, 3), dtype=complex)
        for i in range(3):
            e = np.zeros(3)
            e[i] = step
            fd[:, :, i] = (green.green_paper_sum(d0 + e, w, ALPHA, BETA, RHO)
                           - green.green_paper_sum(d0 - e, w, ALPHA, BETA, RHO)) / (2 * step)
        assert np.abs(dG - fd).max() < 1e-6 * np.abs(dG).max()


def test_tau_moment_series_and_closed_form_agree():
    w = 2 * np.pi * 9.0
    t2 = np.linspace(0.2, 0.8, 13) / w
    t1 = 0.58 * t2
    # evaluate both branches explicitly on either side of the switch
    J = green.tau_moment(w, t1, t2)
    closed = (np.exp(1j * w * t2) * (1 / w**2 - 1j * t2 / w) - np.exp(1j * w * t1) * (1 / w**2 - 1j * t1 / w))
    assert np.allclose(J, closed, rtol=1e-12, atol=0)
