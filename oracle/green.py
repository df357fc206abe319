"""Isotropic background Green's tensor of the LS method (oracle, test infrastructure only).

Time convention e^{-i w t}: outgoing waves carry e^{+i w r / v}, as in A.5.

* ``green_exact``      - the closed-form full-space solution of Eq 7 for an
  isotropic background (Stokes' solution in the frequency domain).  Its two
  1/r terms are exactly the far-field tensor A.5, and its third term tends to
  the near-field tensor A.4 as w -> 0.  This is the default tensor of the
  discrete operator (reading: the paper gives A.4 and A.5 and a near/far
  criterion, A.3, but only their exact combination solves Eq 7).
* ``green_paper_sum``  - A.4 + A.5 evaluated everywhere (the alternative
  reading of Appendix A).
* ``green_self_term``  - the r = 0 cell value: the average of the exact tensor
  over the sphere of volume h^3 centred on the cell, times h^3 (the paper is
  silent on the singular cell).
* ``green_paper_sum_grad`` - the chain-rule derivatives A.6-A.11 of A.4 + A.5,
  written as printed (with E_kl = delta_kl - 3 x_k x_l / r^2, the evident
  reading of the printed "I").

All functions accept a complex ``omega`` (used only by a damped-frequency
physics pin) and broadcast over leading axes of ``d``.
"""

import numpy as np

SPHERE_RADIUS_FACTOR = (3.0 / (4.0 * np.pi)) ** (1.0 / 3.0)


def _radius_and_direction(d):
    d = np.asarray(d, dtype=np.float64)
    r = np.sqrt(np.sum(d * d, axis=-1))
    if np.any(r == 0.0):
        raise ValueError("Green's tensor is singular at r = 0; use green_self_term")
    gam = d / r[..., None]
    return r, gam


def green_exact(d, omega, alpha, beta, rho):
    """G_ij(d) for offsets d[..., 3] (receiver minus source), shape [..., 3, 3].

    G = gg e^{i w r/a}/(4 pi rho a^2 r) + (I - gg) e^{i w r/b}/(4 pi rho b^2 r)
        + (3 gg - I) J(r)/(4 pi rho r^3),
    J(r) = int_{r/a}^{r/b} tau e^{i w tau} dtau = [e^{i w tau}(1/w^2 - i tau/w)]_{r/a}^{r/b}.
    """
    r, g = _radius_and_direction(d)
    w = omega
    gg = g[..., :, None] * g[..., None, :]
    eye = np.eye(3)
    p_term = np.exp(1j * w * r / alpha) / (4.0 * np.pi * rho * alpha**2 * r)
    s_term = np.exp(1j * w * r / beta) / (4.0 * np.pi * rho * beta**2 * r)

    n_term = tau_moment(w, r / alpha, r / beta) / (4.0 * np.pi * rho * r**3)
    return (gg * p_term[..., None, None]
            + (eye - gg) * s_term[..., None, None]
            + (3.0 * gg - eye) * n_term[..., None, None])


SERIES_LIMIT = 0.5   # |w tau| below which the power series replaces the closed forms (cancellation)
SERIES_TERMS = 40


def tau_moment(w, t1, t2):
    """J = int_{t1}^{t2} tau e^{i w tau} dtau.

    Closed form [e^{i w tau}(1/w^2 - i tau/w)]_{t1}^{t2}; where |w t2| < SERIES_LIMIT its two terms
    cancel to O((w t)^2), so the exponential's power series is integrated term by term instead:
    J = sum_n (i w)^n / n! (t2^{n+2} - t1^{n+2}) / (n + 2).
    """
    w = np.asarray(w)
    t1, t2 = np.broadcast_arrays(np.asarray(t1, dtype=np.float64), np.asarray(t2, dtype=np.float64))
    closed = (np.exp(1j * w * t2) * (1.0 / w**2 - 1j * t2 / w)
              - np.exp(1j * w * t1) * (1.0 / w**2 - 1j * t1 / w))
    series = np.zeros(t2.shape, dtype=complex)
    coef = np.ones((), dtype=complex)      # (i w)^n / n!
    p1, p2 = t1**2, t2**2
    for n in range(SERIES_TERMS):
        series = series + coef * (p2 - p1) / (n + 2)
        coef = coef * (1j * w) / (n + 1)
        p1, p2 = p1 * t1, p2 * t2
    return np.where(np.abs(w * t2) < SERIES_LIMIT, series, closed)


def green_paper_sum(d, omega, alpha, beta, rho):
    """A.4 + A.5: G^NF + G^FF at offsets d[..., 3], shape [..., 3, 3]."""
    r, g = _radius_and_direction(d)
    gg = g[..., :, None] * g[..., None, :]
    eye = np.eye(3)
    nf = (-1.0 / (8.0 * np.pi * rho * r * beta**2)) * (1.0 - beta**2 / alpha**2)
    ff_p = np.exp(1j * omega * r / alpha) / (4.0 * np.pi * rho * r * alpha**2)
    ff_s = np.exp(1j * omega * r / beta) / (4.0 * np.pi * rho * r * beta**2)
    return ((eye - 3.0 * gg) * nf[..., None, None]
            + gg * ff_p[..., None, None]
            + (eye - gg) * ff_s[..., None, None])


def sphere_integral(k, a):
    """int_{|x|<a} e^{i k |x|} / (4 pi |x|) dx = int_0^a r e^{i k r} dr = (e^{ika}(1 - ika) - 1)/k^2."""
    return tau_moment(k, 0.0, a)


def green_self_term(h, omega, alpha, beta, rho):
    """Scalar s such that the r = 0 table entry is s * I.

    s = int over the sphere of volume h^3 of G_ii (no sum) = [I(k_p)/(3 a^2) + 2 I(k_s)/(3 b^2)] / rho,
    because the angular average of gg is I/3 and that of (3 gg - I) is 0.
    """
    a = SPHERE_RADIUS_FACTOR * h
    kp = omega / alpha
    ks = omega / beta
    return (sphere_integral(kp, a) / (3.0 * alpha**2)
            + 2.0 * sphere_integral(ks, a) / (3.0 * beta**2)) / rho


def green_paper_sum_grad(d, omega, alpha, beta, rho):
    """dG_kl/dx_i of A.4 + A.5 by the printed chain rule (A.6-A.11); shape [..., 3(k), 3(l), 3(i)]."""
    d = np.asarray(d, dtype=np.float64)
    r = np.sqrt(np.sum(d * d, axis=-1))
    x = d
    eye = np.eye(3)
    xk_xl = x[..., :, None] * x[..., None, :]                      # F_kl
    xk_xl_xi = xk_xl[..., :, :, None] * x[..., None, None, :]
    # (delta_ik x_l + delta_il x_k), indexed [k, l, i]
    dx_sym = np.einsum('ik,...l->...kli', eye, x) + np.einsum('il,...k->...kli', eye, x)
    U = r[..., None, None, None]
    D_i = x[..., None, None, :]
    # near field, A.6-A.7
    C = (1.0 / (8.0 * np.pi * rho * beta**2)) * (1.0 - beta**2 / alpha**2)
    E_kl = (eye - 3.0 * xk_xl / r[..., None, None] ** 2)[..., None]
    g_nf = (C / U**3) * (D_i * E_kl - (3.0 / U**2) * (2.0 * xk_xl_xi - dx_sym * U**2))
    # P far field, A.8-A.9
    X = (np.exp(1j * omega * r / alpha) / (4.0 * np.pi * rho * alpha**2))[..., None, None, None]
    X_i = 1j * omega * X * D_i / (alpha * U)
    Y = (xk_xl / r[..., None, None] ** 2)[..., None]
    Y_i = (U**2 * dx_sym - 2.0 * xk_xl_xi) / U**4
    U_i = D_i / U
    g_p = ((X_i * Y + X * Y_i) * U - X * Y * U_i) / U**2
    # S far field, A.10-A.11
    V = (np.exp(1j * omega * r / beta) / (4.0 * np.pi * rho * beta**2))[..., None, None, None]
    V_i = 1j * omega * V * D_i / (beta * U)
    W = (eye - xk_xl / r[..., None, None] ** 2)[..., None]
    W_i = (-U**2 * dx_sym + 2.0 * xk_xl_xi) / U**4
    g_s = ((V_i * W + V * W_i) * U - V * W * U_i) / U**2
    return g_nf + g_p + g_s
