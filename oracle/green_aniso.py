"""Green's tensor of a homogeneous anisotropic background (oracle, test infrastructure only).

The paper states the method for an arbitrary background (Eq 2-3, 7) but writes out only the
isotropic tensor (Appendix A).  For a general homogeneous background with stiffness c_ijkl and
density rho, the solution of Eq 7 (time convention e^{-i w t}, outgoing waves) is written here
through its plane-wave (unit-sphere) representation, which follows from the Fourier transform
G^(k) = (Gamma(k) - rho w^2 I)^{-1}, Gamma_ik(k) = c_ijkl k_j k_l:

  G(x) = G_s(x) + G_r(x),
  G_s(x) = 1/(8 pi^2 r) * integral over the unit circle n . x = 0 of Gamma(n)^{-1} dphi,
  G_r(x) = i/(8 pi^2) * integral over the half sphere n . x > 0 of
           sum_m P_m(n) k_m(n) / lambda_m(n) * exp(i k_m(n) n . x) dS(n),

with lambda_m(n), P_m(n) the eigenvalues and eigenprojectors of the Christoffel matrix Gamma(n)
(lambda_m = rho v_m^2, the phase velocities of the three modes along n) and k_m = w / v_m.  The
integrand of the full-sphere form is even in n, so the half sphere carries twice its weight.

The zero-offset cell takes, as in the isotropic case, the integral of G over the sphere of
volume h^3 centred on the cell; with the same representation this is the angular mean

  S = 1/(4 pi) * integral over the unit sphere of sum_m P_m(n) I(k_m(n)) / lambda_m(n) dS(n),
  I(k) = integral_0^R r e^{i k r} dr,  R = (3/(4 pi))^{1/3} h,

which for an isotropic background is exactly the sphere-averaged self-term of ``green``.

Quadrature (plain and generous; the integrands are smooth): the half sphere is parametrised about
x^ by u = cos(theta) in [0, 1] (Gauss-Legendre) and the azimuth phi (trapezoid, periodic); the
circle n . x = 0 by the trapezoid rule; the self-term by Gauss-Legendre in cos(theta) over
[-1, 1] times the trapezoid in phi.  The node counts grow with k_max r, the largest phase the
exponential reaches.  The eigen-decomposition is the library routine ``numpy.linalg.eigh``.
"""

import numpy as np
from numpy.polynomial.legendre import leggauss

from . import green as _green

# Voigt index J of the symmetric pair (a, b): 11, 22, 33, 23, 13, 12 (Eq 17)
VOIGT_PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def stiffness4(C):
    """Voigt 6x6 -> c_ijkl [3, 3, 3, 3]."""
    C = np.asarray(C, dtype=np.float64)
    v = np.empty((3, 3), dtype=np.int64)
    for J, (a, b) in enumerate(VOIGT_PAIRS):
        v[a, b] = v[b, a] = J
    c = np.empty((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    c[i, j, k, l] = C[v[i, j], v[k, l]]
    return c


def christoffel(C, n):
    """Gamma_ik(n) = c_ijkl n_j n_l for directions n [..., 3] -> [..., 3, 3]."""
    return np.einsum('ijkl,...j,...l->...ik', stiffness4(C), n, n)


def max_slowness(C, rho, samples=64):
    """max over directions of 1/v (the slowest mode), from a dense sampling of the sphere (10% margin)."""
    t, _ = leggauss(samples)
    phi = 2 * np.pi * np.arange(2 * samples) / (2 * samples)
    T, P = np.meshgrid(t, phi, indexing='ij')
    s = np.sqrt(1 - T**2)
    n = np.stack([s * np.cos(P), s * np.sin(P), T], axis=-1)
    lam = np.linalg.eigvalsh(christoffel(C, n))
    return 1.1 * np.sqrt(rho / lam.min())


def _frame(xhat):
    """Two unit vectors completing x^ to a right-handed orthonormal frame."""
    a = np.zeros(3)
    a[np.argmin(np.abs(xhat))] = 1.0
    e1 = np.cross(xhat, a)
    e1 /= np.linalg.norm(e1)
    return e1, np.cross(xhat, e1)


def node_counts(kr):
    """(n_u, n_phi, n_circle) for a point whose largest phase k_max r is kr."""
    return int(np.ceil(0.3 * kr)) + 36, int(np.ceil(0.3 * kr)) + 72, 128


def _green_points(X, omega, C, rho, n_u, n_phi, n_c):
    """G at the points X [P, 3] (all != 0), with the given node counts -> [P, 3, 3]."""
    r = np.linalg.norm(X, axis=1)
    xhat = X / r[:, None]
    frames = [_frame(x) for x in xhat]
    e1 = np.array([f[0] for f in frames])
    e2 = np.array([f[1] for f in frames])
    # static part: the circle n . x = 0
    phi = 2 * np.pi * np.arange(n_c) / n_c
    nc = np.cos(phi)[None, :, None] * e1[:, None, :] + np.sin(phi)[None, :, None] * e2[:, None, :]
    Gs = np.linalg.inv(christoffel(C, nc)).sum(axis=1) * (2 * np.pi / n_c) / (8 * np.pi**2 * r[:, None, None])
    # regular part: the half sphere n . x > 0, u = n . x^
    t, wt = leggauss(n_u)
    u = 0.5 * (t + 1.0)
    wu = 0.5 * wt
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    s = np.sqrt(1.0 - u**2)
    ring = (np.cos(phi)[None, None, :, None] * e1[:, None, None, :]
            + np.sin(phi)[None, None, :, None] * e2[:, None, None, :])          # [P, 1, n_phi, 3]
    n = u[None, :, None, None] * xhat[:, None, None, :] + s[None, :, None, None] * ring
    lam, V = np.linalg.eigh(christoffel(C, n))                                # [P, n_u, n_phi, 3]
    k = omega * np.sqrt(rho / lam)
    coef = (k / lam) * np.exp(1j * k * r[:, None, None, None] * u[None, :, None, None])
    coef = coef * (wu[None, :, None, None] * (2 * np.pi / n_phi))
    Gr = np.einsum('auqim,auqjm,auqm->aij', V, V, coef) * (1j / (8 * np.pi**2))
    return Gs + Gr


def green_aniso(d, omega, C, rho, scale=1.0, batch=64):
    """G_ij(d) for offsets d[..., 3] != 0 (receiver minus source), shape [..., 3, 3].

    Points that share node counts are evaluated together, ``batch`` at a time; ``scale``
    multiplies every node count (a convergence check)."""
    d = np.asarray(d, dtype=np.float64)
    flat = d.reshape(-1, 3)
    if np.any(np.all(flat == 0.0, axis=1)):
        raise ValueError("Green's tensor is singular at r = 0; use green_aniso_self_term")
    kmax = abs(omega) * max_slowness(C, rho)
    counts = [tuple(int(np.ceil(scale * v)) for v in node_counts(kmax * np.linalg.norm(x))) for x in flat]
    out = np.empty((flat.shape[0], 3, 3), dtype=complex)
    groups = {}
    for p, cnt in enumerate(counts):
        groups.setdefault(cnt, []).append(p)
    for cnt, idx in groups.items():
        for b in range(0, len(idx), batch):
            sel = np.array(idx[b:b + batch])
            out[sel] = _green_points(flat[sel], omega, C, rho, *cnt)
    return out.reshape(d.shape[:-1] + (3, 3))


def green_aniso_self_term(h, omega, C, rho, n_t=48, n_phi=96):
    """S [3, 3] = integral of G over the sphere of volume h^3 centred on the source (the r = 0 cell)."""
    a = _green.SPHERE_RADIUS_FACTOR * h
    t, wt = leggauss(n_t)
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    s = np.sqrt(1.0 - t**2)
    n = np.stack([s[:, None] * np.cos(phi)[None, :], s[:, None] * np.sin(phi)[None, :],
                  np.broadcast_to(t[:, None], (n_t, n_phi))], axis=-1)
    lam, V = np.linalg.eigh(christoffel(C, n))
    k = omega * np.sqrt(rho / lam)
    coef = _green.sphere_integral(k, a) / lam
    w = wt[:, None] * (2 * np.pi / n_phi) / (4 * np.pi)
    return np.einsum('tpim,tpjm,tpm,tp->ij', V, V, coef, w)
