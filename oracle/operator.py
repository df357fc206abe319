"""The discrete LS displacement operator, written out plainly (oracle, test infrastructure only).

Discretisation (the readings are listed with each function):

* grid: cell centres x = (i, j, k) h, 0 <= i < N1 (x), j < N2 (y), k < N3 (z);
  arrays are stored [z][y][x] (numpy C order of (N3, N2, N1)).
* strain (Eq 17-18): Voigt engineering strain eps = E u with second-order central
  differences inside and the first-order one-sided difference (forward at index
  0, backward at index N-1) on the model boundary.
* contrast (Eq 8, 11-12): Voigt stress tau = dC eps per cell; the term
  [dC u_,]_,k of Eq 5 is the divergence of tau, taken as -E^T tau (the exact
  discrete adjoint of the strain stencil; reading of the k-space H of Eq 21).
  B = -E^T dC E + w^2 drho, acting on u.
* Green's operator: linear (non-periodic) convolution with the table
  T(m) = h^3 G(m h) for m != 0 and T(0) = the sphere-averaged self-term.
* A = I - Gconv B  (Eq 19-21 left side); the incident field of a moment tensor
  M at cell s (Eq 13-16, Aki-Richards sign) is b = e^{i w t0} Gconv E^T (M delta_s) / h^3.
* background: if C0 is not isotropic, the isotropic reference takes
  c11 = C33, c44 = (C44 + C55)/2 (the rule of the paper's Model 1) and C0 - C_iso
  is added to the contrast of every cell.  Mode 'aniso' instead convolves with the
  Green's tensor of C0 itself (``green_aniso``) and adds nothing to the contrast.
"""

import numpy as np
import scipy.sparse as sp

from . import green as _green
from . import green_aniso as _green_aniso

# Voigt index J -> tensor pair (0-based x, y, z): 11, 22, 33, 23, 13, 12 (Eq 17)
VOIGT_PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))
# packing order of the 21 upper-triangle values of a symmetric 6x6
UPPER21 = tuple((I, J) for I in range(6) for J in range(I, 6))


def voigt_index(a, c):
    """Voigt index of the symmetric tensor pair (a, c)."""
    for J, (p, q) in enumerate(VOIGT_PAIRS):
        if (p, q) == (a, c) or (q, p) == (a, c):
            return J
    raise ValueError((a, c))


def unpack21(dc21):
    """[21, ...] packed upper triangle -> [6, 6, ...] symmetric."""
    dc21 = np.asarray(dc21)
    out = np.zeros((6, 6) + dc21.shape[1:], dtype=dc21.dtype)
    for n, (I, J) in enumerate(UPPER21):
        out[I, J] = dc21[n]
        out[J, I] = dc21[n]
    return out


def pack21(c66):
    c66 = np.asarray(c66)
    return np.stack([c66[I, J] for (I, J) in UPPER21])


def iso_stiffness(c11, c44):
    """Isotropic Voigt stiffness with C12 = C11 - 2 C44."""
    c12 = c11 - 2.0 * c44
    C = np.zeros((6, 6))
    C[:3, :3] = c12
    for I in range(3):
        C[I, I] = c11
        C[I + 3, I + 3] = c44
    return C


def is_isotropic(C0, rtol=1e-12):
    C0 = np.asarray(C0, dtype=np.float64)
    ref = iso_stiffness(C0[0, 0], C0[3, 3])
    return np.all(np.abs(C0 - ref) <= rtol * np.abs(C0).max())


def iso_reference(C0, rho0):
    """(alpha, beta, C_iso): the isotropic reference medium and its velocities (Eq 2-3)."""
    C0 = np.asarray(C0, dtype=np.float64)
    if is_isotropic(C0):
        c11, c44 = C0[0, 0], C0[3, 3]
    else:
        c11, c44 = C0[2, 2], 0.5 * (C0[3, 3] + C0[4, 4])
    return np.sqrt(c11 / rho0), np.sqrt(c44 / rho0), iso_stiffness(c11, c44)


def total_contrast21(C0, rho0, dc21):
    """Per-cell contrast with the anisotropic part of the background folded in."""
    _, _, c_iso = iso_reference(C0, rho0)
    fold = pack21(np.asarray(C0, dtype=np.float64) - c_iso)
    return np.asarray(dc21, dtype=np.float64) + fold.reshape((21,) + (1,) * (np.ndim(dc21) - 1))


def taper_weights(shape, d):
    """Absorbing-boundary weight of every cell (Eq 23-25): 1 - exp(-l^2 / (N_a h^2)) inside the boundary
    layer, 1 elsewhere.  Readings (the paper leaves them open): the layer is the cells within d cells of a
    face; x_L is where the ray from the model centre through the cell centre leaves the box, whose faces
    lie half a cell outside the outer cell centres; l = |x_L - x_B|; N_a is the number of cells along the
    axis a whose face the ray crosses.  Lengths in cells (h cancels).  shape (N1, N2, N3) -> [N3, N2, N1]."""
    n = np.array(shape, dtype=np.int64)
    w = np.ones((n[2], n[1], n[0]))
    if d <= 0:
        return w
    centre = (n - 1) / 2.0
    for k in range(n[2]):
        for j in range(n[1]):
            for i in range(n[0]):
                p = np.array([i, j, k], dtype=np.float64)
                if all(d <= p[a] <= n[a] - 1 - d for a in range(3)):
                    continue                          # not in the layer
                v = p - centre
                best, axis = np.inf, -1
                for a in range(3):
                    if v[a] == 0.0:
                        continue
                    face = n[a] - 0.5 if v[a] > 0 else -0.5
                    s_ = (face - centre[a]) / v[a]   # ray parameter of the face crossing
                    if s_ < best:
                        best, axis = s_, a
                if axis < 0:
                    continue                          # the centre itself
                l = (best - 1.0) * np.linalg.norm(v)
                w[k, j, i] = 1.0 - np.exp(-l * l / n[axis])
    return w


# ----------------------------------------------------------------------------------------------
# strain stencil (Eq 18)


def deriv_1d(n, h):
    """n x n matrix of d/dx: (u[i+1]-u[i-1])/2h inside, (u[1]-u[0])/h and (u[n-1]-u[n-2])/h at the ends."""
    if n < 2:
        raise ValueError("a derivative needs at least 2 cells along each axis")
    D = np.zeros((n, n))
    for i in range(1, n - 1):
        D[i, i + 1] = 1.0 / (2.0 * h)
        D[i, i - 1] = -1.0 / (2.0 * h)
    D[0, 0], D[0, 1] = -1.0 / h, 1.0 / h
    D[n - 1, n - 1], D[n - 1, n - 2] = 1.0 / h, -1.0 / h
    return D


def deriv_op(shape, h, axis):
    """Sparse d/dx_axis on the flattened [z][y][x] grid; shape = (N1, N2, N3), axis 0=x, 1=y, 2=z."""
    n1, n2, n3 = shape
    eyes = [sp.identity(n3, format='csr'), sp.identity(n2, format='csr'), sp.identity(n1, format='csr')]
    factors = list(eyes)
    factors[2 - axis] = sp.csr_matrix(deriv_1d(shape[axis], h))
    return sp.kron(factors[0], sp.kron(factors[1], factors[2]), format='csr')


def strain_operator(shape, h):
    """Sparse E (6n x 3n): eps_J = sum over pairs (a, c) with voigt_index(a, c) = J of d_a u_c."""
    D = [deriv_op(shape, h, a) for a in range(3)]
    blocks = [[None] * 3 for _ in range(6)]
    for a in range(3):
        for c in range(3):
            J = voigt_index(a, c)
            blocks[J][c] = D[a] if blocks[J][c] is None else blocks[J][c] + D[a]
    n = shape[0] * shape[1] * shape[2]
    for J in range(6):
        for c in range(3):
            if blocks[J][c] is None:
                blocks[J][c] = sp.csr_matrix((n, n))
    return sp.bmat(blocks, format='csr')


def strain_apply(u, h):
    """eps = E u by array slicing (same stencil as strain_operator); u [3, N3, N2, N1] -> [6, N3, N2, N1]."""
    def d(f, axis):
        ax = 2 - axis
        f = np.moveaxis(f, ax, 0)
        out = np.empty_like(f)
        out[1:-1] = (f[2:] - f[:-2]) / (2.0 * h)
        out[0] = (f[1] - f[0]) / h
        out[-1] = (f[-1] - f[-2]) / h
        return np.moveaxis(out, 0, ax)
    eps = np.zeros((6,) + u.shape[1:], dtype=np.result_type(u, np.float64))
    for a in range(3):
        for c in range(3):
            eps[voigt_index(a, c)] += d(u[c], a)
    return eps


def strain_adjoint_apply(tau, h):
    """E^T tau by array slicing; tau [6, N3, N2, N1] -> [3, N3, N2, N1]."""
    def dt(v, axis):
        ax = 2 - axis
        v = np.moveaxis(v, ax, 0)
        out = np.zeros_like(v)
        out[2:] += v[1:-1] / (2.0 * h)
        out[:-2] -= v[1:-1] / (2.0 * h)
        out[0] -= v[0] / h
        out[1] += v[0] / h
        out[-1] += v[-1] / h
        out[-2] -= v[-1] / h
        return np.moveaxis(out, 0, ax)
    f = np.zeros((3,) + tau.shape[1:], dtype=np.result_type(tau, np.float64))
    for a in range(3):
        for c in range(3):
            f[c] += dt(tau[voigt_index(a, c)], a)
    return f


# ----------------------------------------------------------------------------------------------
# contrast operator B


def contrast_operator(shape, h, dc21_total, drho, omega):
    """Sparse B = -E^T dC E + w^2 drho (3n x 3n); dc21_total already includes the folded background."""
    n = shape[0] * shape[1] * shape[2]
    E = strain_operator(shape, h)
    c66 = unpack21(np.asarray(dc21_total).reshape(21, n))
    C = sp.bmat([[sp.diags(c66[I, J]) for J in range(6)] for I in range(6)], format='csr')
    R = sp.kron(sp.identity(3), sp.diags(np.asarray(drho).reshape(n)), format='csr')
    return -(E.T @ C @ E) + omega**2 * R


def contrast_apply(u, h, dc21_total, drho, omega):
    """B u by array slicing; u [3, N3, N2, N1]."""
    eps = strain_apply(u, h)
    tau = np.einsum('IJ...,J...->I...', unpack21(dc21_total), eps)
    return -strain_adjoint_apply(tau, h) + omega**2 * drho[None] * u


# ----------------------------------------------------------------------------------------------
# Green's table and convolution


def green_tensor(d, omega, alpha, beta, rho, mode, C0=None):
    if mode == 'exact':
        return _green.green_exact(d, omega, alpha, beta, rho)
    if mode == 'paper_sum':
        return _green.green_paper_sum(d, omega, alpha, beta, rho)
    if mode == 'aniso':
        return _green_aniso.green_aniso(d, omega, C0, rho)
    raise ValueError(mode)


def self_matrix(h, omega, alpha, beta, rho, mode, C0=None):
    """The r = 0 table entry (a 3x3 matrix): the integral of G over the sphere of volume h^3."""
    if mode == 'aniso':
        return _green_aniso.green_aniso_self_term(h, omega, C0, rho)
    return _green.green_self_term(h, omega, alpha, beta, rho) * np.eye(3)


def green_table(shape, h, omega, alpha, beta, rho, mode='exact', C0=None):
    """T[3, 3, 2N3-1, 2N2-1, 2N1-1]: T at offset (dx, dy, dz) stored at [..., dz+N3-1, dy+N2-1, dx+N1-1]."""
    n1, n2, n3 = shape
    oz, oy, ox = np.meshgrid(np.arange(-(n3 - 1), n3), np.arange(-(n2 - 1), n2),
                             np.arange(-(n1 - 1), n1), indexing='ij')
    d = np.stack([ox, oy, oz], axis=-1).astype(np.float64) * h
    zero = (ox == 0) & (oy == 0) & (oz == 0)
    d[zero] = 1.0  # placeholder, overwritten below
    if mode == 'aniso':
        # G(-x) = G(x) for every homogeneous medium (Gamma(n) is even in n): evaluate the half of the
        # offsets that comes first in (dz, dy, dx) order, then mirror it through the origin
        half = (oz > 0) | ((oz == 0) & (oy > 0)) | ((oz == 0) & (oy == 0) & (ox > 0))
        G = np.zeros(d.shape[:-1] + (3, 3), dtype=complex)
        G[half] = green_tensor(d[half], omega, alpha, beta, rho, mode, C0) * h**3
        G = G + G[::-1, ::-1, ::-1]
    else:
        G = green_tensor(d, omega, alpha, beta, rho, mode) * h**3
    G[zero] = self_matrix(h, omega, alpha, beta, rho, mode, C0)
    return np.moveaxis(G, (-2, -1), (0, 1))


def cell_coords(shape):
    n1, n2, n3 = shape
    k, j, i = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing='ij')
    return np.stack([i.ravel(), j.ravel(), k.ravel()], axis=-1)


def dense_green(shape, T):
    """Dense Gconv (3n x 3n): Gconv[(i,p),(j,q)] = T_ij(p - q)."""
    n1, n2, n3 = shape
    P = cell_coords(shape)
    off = P[:, None, :] - P[None, :, :]
    blk = T[:, :, off[..., 2] + n3 - 1, off[..., 1] + n2 - 1, off[..., 0] + n1 - 1]  # [3,3,n,n]
    n = P.shape[0]
    return blk.transpose(0, 2, 1, 3).reshape(3 * n, 3 * n)


def convolve_at(f, shape, h, omega, alpha, beta, rho, cells, mode='exact', C0=None):
    """(Gconv f) at the listed cells by direct O(n) sums per cell; f [3, N3, N2, N1]; cells [m, 3] (x,y,z)."""
    P = cell_coords(shape)
    fv = f.reshape(3, -1)
    out = np.zeros((len(cells), 3), dtype=complex)
    self_val = self_matrix(h, omega, alpha, beta, rho, mode, C0)
    for t, c in enumerate(np.asarray(cells)):
        d = (c[None, :] - P).astype(np.float64) * h
        here = np.all(d == 0.0, axis=1)
        d[here] = 1.0
        G = green_tensor(d, omega, alpha, beta, rho, mode, C0) * h**3
        G[here] = self_val
        out[t] = np.einsum('qij,jq->i', G, fv)
    return out


def convolve_fft(f, T):
    """Gconv f by zero-padded FFT (2N per axis); equals dense_green(T) @ f (a library FFT as the step)."""
    import scipy.fft as sfft
    n3, n2, n1 = f.shape[1:]
    shp = (2 * n3, 2 * n2, 2 * n1)
    Tp = np.zeros((3, 3) + shp, dtype=complex)
    idx = [np.arange(-(n - 1), n) % (2 * n) for n in (n3, n2, n1)]
    Tp[:, :, idx[0][:, None, None], idx[1][None, :, None], idx[2][None, None, :]] = T
    That = sfft.fftn(Tp, axes=(2, 3, 4), workers=-1)
    fp = np.zeros((3,) + shp, dtype=complex)
    fp[:, :n3, :n2, :n1] = f
    fhat = sfft.fftn(fp, axes=(1, 2, 3), workers=-1)
    vhat = np.einsum('ij...,j...->i...', That, fhat)
    return sfft.ifftn(vhat, axes=(1, 2, 3), workers=-1)[:, :n3, :n2, :n1]


# ----------------------------------------------------------------------------------------------
# the operator and its right-hand sides


class Problem:
    """One (grid, medium, frequency) instance of the discrete LS system."""

    def __init__(self, shape, h, C0, rho0, dc21, drho, omega, mode='exact', taper=0):
        self.shape = tuple(int(v) for v in shape)
        self.h = float(h)
        self.omega = omega
        self.rho0 = float(rho0)
        self.alpha, self.beta, self.c_iso = iso_reference(C0, rho0)
        self.C0 = np.asarray(C0, dtype=np.float64)
        n3, n2, n1 = self.shape[2], self.shape[1], self.shape[0]
        w = taper_weights(self.shape, taper)   # the absorbing layer weights the total contrast (Eq 25)
        dc21 = np.asarray(dc21, dtype=np.float64).reshape(21, n3, n2, n1)
        if mode != 'aniso':
            dc21 = total_contrast21(C0, rho0, dc21)
        self.dc21 = dc21 * w[None]
        self.drho = np.asarray(drho, dtype=np.float64).reshape(n3, n2, n1) * w
        self.mode = mode
        self._T = None

    @property
    def n(self):
        return self.shape[0] * self.shape[1] * self.shape[2]

    @property
    def field_shape(self):
        return (3, self.shape[2], self.shape[1], self.shape[0])

    def table(self):
        if self._T is None:
            self._T = green_table(self.shape, self.h, self.omega, self.alpha, self.beta, self.rho0, self.mode,
                                  self.C0)
        return self._T

    def B(self):
        return contrast_operator(self.shape, self.h, self.dc21, self.drho, self.omega)

    def dense_A(self):
        Gd = dense_green(self.shape, self.table())
        return np.eye(3 * self.n) - Gd @ self.B().toarray()

    def contrast(self, u):
        return contrast_apply(u, self.h, self.dc21, self.drho, self.omega)

    def apply_fft(self, u):
        """A u via the zero-padded FFT convolution (secondary reference T2)."""
        return u - convolve_fft(self.contrast(u), self.table())

    def apply_bruteforce(self, u, cells=None):
        """A u by direct summation; full field, or only the listed cells ([m, 3] x,y,z) -> [m, 3]."""
        f = self.contrast(u)
        if cells is None:
            v = (dense_green(self.shape, self.table()) @ f.reshape(-1)).reshape(u.shape)
            return u - v
        cells = np.asarray(cells)
        v = convolve_at(f, self.shape, self.h, self.omega, self.alpha, self.beta, self.rho0, cells, self.mode,
                        self.C0)
        return u[:, cells[:, 2], cells[:, 1], cells[:, 0]].T - v

    def moment_source(self, M, src):
        """E^T (M delta_s) / h^3 as a force density [3, N3, N2, N1]; M Voigt (11,22,33,23,13,12)."""
        tau = np.zeros((6,) + self.field_shape[1:])
        i, j, k = src
        tau[:, k, j, i] = np.asarray(M, dtype=np.float64)
        return strain_adjoint_apply(tau, self.h) / self.h**3

    def convolve_point_sources(self, f):
        """Gconv f for a force density f with few non-zero cells, by direct closed-form sums over all cells.

        The anisotropic tensor has no closed form; mode 'aniso' convolves with the sampled table instead."""
        if self.mode == 'aniso':
            return convolve_fft(f, self.table())
        P = cell_coords(self.shape)
        out = np.zeros((self.n, 3), dtype=complex)
        self_val = self_matrix(self.h, self.omega, self.alpha, self.beta, self.rho0, self.mode, self.C0)
        fv = f.reshape(3, -1)
        for q in np.flatnonzero(np.any(fv != 0, axis=0)):
            d = (P - P[q][None, :]).astype(np.float64) * self.h
            here = np.all(d == 0.0, axis=1)
            d[here] = 1.0
            G = green_tensor(d, self.omega, self.alpha, self.beta, self.rho0, self.mode, self.C0) * self.h**3
            G[here] = self_val
            out += G @ fv[:, q]
        return out.T.reshape(self.field_shape)

    def rhs_moment(self, M, src, t0=0.0):
        """Incident field b = e^{i w t0} Gconv E^T (M delta_s) / h^3, by direct closed-form sums (Eq 13-16)."""
        return np.exp(1j * self.omega * t0) * self.convolve_point_sources(self.moment_source(M, src))

    def rhs_force(self, F, cell):
        """Incident field of a point force F delta_cell / h^3: b = Gconv (F delta) / h^3 (Eq 6)."""
        f = np.zeros(self.field_shape, dtype=complex)
        i, j, k = cell
        f[:, k, j, i] = np.asarray(F, dtype=np.float64) / self.h**3
        return self.convolve_point_sources(f)
