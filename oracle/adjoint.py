"""Transposed operator and misfit gradients by dense linear algebra (oracle, test infrastructure only).

Definitions:
* A^T: Gconv is symmetric (the Green's tensor is symmetric and even) and so is B, hence
  A^T = I - B Gconv; ``apply_T`` uses that form and ``dense_A().T`` is the definition it is tested against.
* Misfit J = 1/2 sum over frequencies and sources of ||P u - d||^2 with P the selection of the three
  components at receiver cells, u = A^{-1} b(M, s).
* ``misfit_gradient_dense`` computes J and dJ/dtheta for the packed contrast (21 per cell), the
  density contrast and the moment tensors by the adjoint method with dense matrices:
  lambda = A^{-H} P^H (P u - d),  mu = Gconv^H lambda,
  dJ/d dC_JK(x) = -Re[conj(eps_J(mu)) eps_K(u) + (J != K) conj(eps_K(mu)) eps_J(u)](x),
  dJ/d drho(x)  = w^2 Re[sum_c conj(mu_c) u_c](x),
  dJ/d M_J      = Re[e^{i w t0} conj(eps_J(mu)(s))] / h^3.
  It is pinned against central finite differences of J computed with dense LU solves.
"""

import numpy as np

from . import operator as op


def apply_T(P, y):
    """A^T y = y - B (Gconv y) through the zero-padded FFT convolution."""
    return y - P.contrast(op.convolve_fft(y, P.table()))


def receiver_sample(u, receivers):
    r = np.asarray(receivers)
    return u[:, r[:, 2], r[:, 1], r[:, 0]]


def misfit(problems, sources, receivers, data):
    """J and the forward fields; problems: one Problem per frequency; sources: [(M, s, t0)];
    data[iw][isrc]: complex [3, nrec]."""
    J = 0.0
    fields = []
    for iw, P in enumerate(problems):
        A = P.dense_A()
        us = []
        for isrc, (M, s, t0) in enumerate(sources):
            u = np.linalg.solve(A, P.rhs_moment(M, s, t0).reshape(-1)).reshape(P.field_shape)
            r = receiver_sample(u, receivers) - data[iw][isrc]
            J += 0.5 * np.vdot(r, r).real
            us.append(u)
        fields.append(us)
    return J, fields


def misfit_gradient_dense(problems, sources, receivers, data):
    """(J, g21 [21, N3, N2, N1], grho [N3, N2, N1], gM [nsrc, 6]) by the dense adjoint method."""
    P0 = problems[0]
    g21 = np.zeros((21,) + P0.field_shape[1:])
    grho = np.zeros(P0.field_shape[1:])
    gM = np.zeros((len(sources), 6))
    J = 0.0
    rec = np.asarray(receivers)
    h3 = P0.h**3
    for P in problems:
        A = P.dense_A()
        Gd = op.dense_green(P.shape, P.table())
        for isrc, (M, s, t0) in enumerate(sources):
            iw = problems.index(P)
            u = np.linalg.solve(A, P.rhs_moment(M, s, t0).reshape(-1)).reshape(P.field_shape)
            r = receiver_sample(u, receivers) - data[iw][isrc]
            J += 0.5 * np.vdot(r, r).real
            adj_src = np.zeros(P.field_shape, dtype=complex)
            adj_src[:, rec[:, 2], rec[:, 1], rec[:, 0]] = r
            lam = np.linalg.solve(A.conj().T, adj_src.reshape(-1))
            mu = (Gd.conj().T @ lam).reshape(P.field_shape)
            eu = op.strain_apply(u, P.h)
            em = op.strain_apply(mu, P.h)
            for n, (I, K) in enumerate(op.UPPER21):
                v = (np.conj(em[I]) * eu[K]).real
                if I != K:
                    v = v + (np.conj(em[K]) * eu[I]).real
                g21[n] -= v
            grho += (P.omega**2) * np.sum(np.conj(mu) * u, axis=0).real
            i, j, k = s
            gM[isrc] += (np.exp(1j * P.omega * t0) * np.conj(em[:, k, j, i])).real / h3
    return J, g21, grho, gM


VTI_NAMES = ("C11", "C33", "C44", "C66", "C13")


def vti_chain(g21):
    """Gradient for the 5 VTI parameters per cell (C22 = C11, C55 = C44, C23 = C13, C12 = C11 - 2 C66)
    from the gradient for the 21 packed entries."""
    idx = {pair: n for n, pair in enumerate(op.UPPER21)}
    g = lambda I, J: g21[idx[(I, J)]]
    return np.stack([g(0, 0) + g(1, 1) + g(0, 1),
                     g(2, 2),
                     g(3, 3) + g(4, 4),
                     g(5, 5) - 2.0 * g(0, 1),
                     g(0, 2) + g(1, 2)])
