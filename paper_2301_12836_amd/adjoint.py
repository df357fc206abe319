"""Gradients of a receiver misfit through the LS solve, as a torch.autograd.Function.

Forward: for every frequency, the incident fields of the moment-tensor sources (Eq 13-16) and one
batched solve A u = u0 (Eq 21-22); the fields are kept per frequency (checkpoints, held by the autograd
node together with a copy of the medium, which backward restores on the context) and the three
components at the receiver cells are returned, complex [n_freq, n_src, 3, n_rec].

Backward (adjoint-state method): with g = dL/d(data) (PyTorch's convention: for L = 1/2 ||data - d||^2
it is the residual data - d), per frequency
  A^T lambda_bar = conj(P^H g)         (ls_solve_T; A^H lambda = P^H g with lambda_bar = conj(lambda))
  then, in one ls_grad call:
  mu = conj(Gconv lambda_bar)
  dL/d dC, dL/d drho                   (accumulated over frequencies and sources)
  dL/d M_J = Re[e^{i w t0} conj(eps_J(mu)(s))] / h^3   (strain of mu at the source cell)
because dA = -Gconv dB, du0/dM_J = e^{i w t0} Gconv E^T (e_J delta_s)/h^3 and Gconv^H = conj(Gconv).
All field work runs in the HIP library; torch only gathers receiver values and adds small arrays.
"""

import numpy as np
import torch

from . import lsvie

UPPER21 = tuple((I, J) for I in range(6) for J in range(I, 6))


class MisfitSetup:
    """A context plus the acquisition: sources [(M6, (i, j, k), t0)], receivers [n_rec, 3] cells."""

    def __init__(self, ctx, source_cells, receivers, t0=None, tol=1e-10, maxit=3000, precision="c128"):
        self.ctx = ctx
        self.source_cells = [tuple(int(v) for v in s) for s in source_cells]
        self.t0 = [0.0] * len(self.source_cells) if t0 is None else [float(v) for v in t0]
        rec = np.asarray(receivers, dtype=np.int64)
        self.rec = rec
        dev = ctx.device
        self.ri = torch.as_tensor(rec[:, 0], device=dev)
        self.rj = torch.as_tensor(rec[:, 1], device=dev)
        self.rk = torch.as_tensor(rec[:, 2], device=dev)
        self.tol = tol
        self.maxit = maxit
        self.precision = precision
        self.fields = None
        self.infos = None

    @property
    def n_src(self):
        return len(self.source_cells)

    def sample(self, u):
        return u[:, :, self.rk, self.rj, self.ri]


class _LSData(torch.autograd.Function):
    @staticmethod
    def forward(fctx, dc21, drho, M, setup):
        ctx = setup.ctx
        ctx.set_contrast(dc21.detach(), drho.detach())
        Mh = M.detach().cpu().numpy().astype(np.float64)
        fields, out, infos = [], [], []
        for iw in range(len(ctx.omegas)):
            b = torch.stack([ctx.rhs_moment(Mh[s], setup.source_cells[s], i_omega=iw, t0=setup.t0[s])
                             for s in range(setup.n_src)])
            u, inf = ctx.solve(b, i_omega=iw, tol=setup.tol, maxit=setup.maxit, precision=setup.precision)
            fields.append(u)
            infos.append(inf)
            out.append(setup.sample(u))
        setup.fields = fields
        setup.infos = infos
        # the checkpoints and the medium belong to this node: another forward on the same setup before
        # this node's backward must not change what its backward sees
        fctx.setup = setup
        fctx.fields = fields
        fctx.medium = (dc21.detach().clone(), drho.detach().clone())
        return torch.stack(out)

    @staticmethod
    def backward(fctx, g):
        setup = fctx.setup
        ctx = setup.ctx
        ctx.set_contrast(*fctx.medium)   # the adjoint operator and the gradient need this node's medium
        g21 = torch.zeros((21,) + ctx.field_shape[1:], dtype=torch.float64, device=ctx.device)
        grho = torch.zeros(ctx.field_shape[1:], dtype=torch.float64, device=ctx.device)
        gM = torch.zeros((setup.n_src, 6), dtype=torch.float64, device=ctx.device)
        for iw, w in enumerate(ctx.omegas):
            adj = torch.zeros((setup.n_src,) + ctx.field_shape, dtype=torch.complex128, device=ctx.device)
            for s in range(setup.n_src):
                comp = adj[s]
                for c in range(3):
                    comp[c].index_put_((setup.rk, setup.rj, setup.ri), g[iw, s, c].conj().to(torch.complex128),
                                       accumulate=True)
            lam_bar, _ = ctx.solve_T(adj, i_omega=iw, tol=setup.tol, maxit=setup.maxit, precision=setup.precision)
            # one library call: mu = conj(Gconv lam_bar), then the dC, drho and moment-tensor gradients
            _, _, gMw = ctx.grad(fctx.fields[iw], lam_bar, i_omega=iw, src=setup.source_cells, t0=setup.t0,
                                 g_dC=g21, g_drho=grho)
            gM += torch.from_numpy(gMw).to(gM.device)
        return g21, grho, gM.to(torch.float64), None


def receiver_data(dc21, drho, M, setup):
    """Differentiable receiver data, complex [n_freq, n_src, 3, n_rec]."""
    return _LSData.apply(dc21, drho, M, setup)


def misfit(dc21, drho, M, setup, observed):
    """L = 1/2 sum |data - observed|^2 (real scalar, differentiable)."""
    r = receiver_data(dc21, drho, M, setup) - observed
    return 0.5 * torch.sum(r.real ** 2 + r.imag ** 2)


def vti_from_packed_grad(g21):
    """Chain rule to (C11, C33, C44, C66, C13) per cell with C22 = C11, C55 = C44, C23 = C13,
    C12 = C11 - 2 C66: returns [5, N3, N2, N1]."""
    idx = {pair: n for n, pair in enumerate(UPPER21)}
    g = lambda I, J: g21[idx[(I, J)]]
    return torch.stack([g(0, 0) + g(1, 1) + g(0, 1), g(2, 2), g(3, 3) + g(4, 4), g(5, 5) - 2.0 * g(0, 1),
                        g(0, 2) + g(1, 2)])


def vti_to_packed(p5, base21):
    """Packed 21-contrast from per-cell VTI contrasts (dC11, dC33, dC44, dC66, dC13) added to base21."""
    idx = {pair: n for n, pair in enumerate(UPPER21)}
    out = base21.clone()
    c11, c33, c44, c66, c13 = p5
    out[idx[(0, 0)]] += c11
    out[idx[(1, 1)]] += c11
    out[idx[(0, 1)]] += c11 - 2.0 * c66
    out[idx[(2, 2)]] += c33
    out[idx[(3, 3)]] += c44
    out[idx[(4, 4)]] += c44
    out[idx[(5, 5)]] += c66
    out[idx[(0, 2)]] += c13
    out[idx[(1, 2)]] += c13
    return out
