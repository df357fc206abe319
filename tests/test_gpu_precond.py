"""GPU parity of the block-Jacobi preconditioner (ls_options.precond = LS_PRECOND_BLOCK_JACOBI) against the
oracle (``oracle.precond``, pinned in test_oracle_precond.py).

* the inverse diagonal blocks equal the inverses of the oracle's blocks, at every cell of small grids
  (boundary, edge and corner cells included, an axis of two cells too) and at sampled cells of 128^3 grids,
  with the closed-form Green's tensor and the anisotropic octant and half-space tables; FP64, relative
  1e-12 (closed form) and 1e-9 (the anisotropic tables, which agree with the oracle's to 1e-10);
* ls_set_contrast rebuilds them;
* preconditioned solves, FP64 and mixed, forward and transposed, at one and at several frequencies in one
  call, reach the dense LU solution (1e-10 / 1e-5), and a system in a multi-frequency solve is bitwise its
  solo solve;
* on a strongly heterogeneous medium the preconditioner cuts the matvecs (the oracle's right-preconditioned
  Bi-CGSTAB takes about a third fewer there).
"""

import numpy as np
import pytest

from oracle import operator as op, precond, solve
from paper_2301_12836_amd import models

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2301_12836_amd import lsvie  # noqa: E402

H = 10.0
WS = [2 * np.pi * 15.0, 2 * np.pi * 31.0]
C_ORTHO, RHO_ORTHO = models.ortho_background()
C_TTI = models.tti_cfg3()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def medium(shape, seed, rel_=0.2, background=None):
    m = models.random_medium(shape, seed, rel=rel_, h=H, aniso_background=background == "vti")
    if background == "ortho":
        m.C0, m.rho0 = np.asarray(C_ORTHO), float(RHO_ORTHO)
    elif background == "tti":
        m.C0 = np.asarray(C_TTI)
    return m


def block_err(got, D):
    """max over cells of |got - D^-1| / max |D^-1| (got [.., 3, 3] from the library)."""
    want = np.linalg.inv(D)
    return float(np.abs(got.reshape(-1, 3, 3) - want).max() / np.abs(want).max())


@pytest.mark.parametrize("shape,mode,background,bar", [
    ((6, 5, 7), "exact", None, 1e-12),
    ((5, 6, 4), "exact", "vti", 1e-12),
    ((2, 5, 6), "paper_sum", "vti", 1e-12),
    ((6, 5, 4), "aniso", "ortho", 1e-9),
    ((5, 4, 6), "aniso", "tti", 1e-9),
])
def test_blocks_match_oracle(shape, mode, background, bar):
    m = medium(shape, 31, background=background)
    ctx = lsvie.context_from_model(m, omegas=WS, precision="mixed", green_mode=mode, precond="block_jacobi")
    for iw, w in enumerate(WS):
        P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, w, mode=mode)
        D = precond.block_diagonal(P)
        e = block_err(ctx.precond_blocks(iw).cpu().numpy(), D)
        print(shape, mode, background, "freq", iw, "inverse blocks vs oracle", e, flush=True)
        assert e < bar
    ctx.close()


def test_set_contrast_rebuilds_blocks():
    m = medium((7, 6, 5), 32, background="vti")
    ctx = lsvie.context_from_model(m, omegas=WS[:1], precision="c128", precond="block_jacobi")
    m2 = medium((7, 6, 5), 33, rel_=0.3, background="vti")
    ctx.set_contrast(m2.dc21, m2.drho)
    P = op.Problem(m.shape, m.h, m.C0, m.rho0, m2.dc21, m2.drho, WS[0])
    e = block_err(ctx.precond_blocks(0).cpu().numpy(), precond.block_diagonal(P))
    print("after set_contrast", e, flush=True)
    assert e < 1e-12
    ctx.close()


def test_preconditioned_solves_match_dense():
    m = medium((7, 6, 5), 34, rel_=0.3, background="vti")
    ctx = lsvie.context_from_model(m, omegas=WS, precision="mixed", max_rhs=2, precond="block_jacobi")
    P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, WS[1])
    A = P.dense_A()
    b = np.stack([P.rhs_moment(models.double_couple(30, 60, 90), (3, 2, 1)), models.random_field(m.shape, 5)])
    want = np.stack([solve.solve_dense(A, b[q]) for q in range(2)])
    bt = torch.from_numpy(b)
    x, inf = ctx.solve(bt, i_omega=1, tol=1e-12, maxit=1000, precision="c128")
    xm, infm = ctx.solve(bt, i_omega=1, tol=1e-7, maxit=1000, precision="mixed")
    for q in range(2):
        print("system", q, "c128", inf[q], rel(x[q].cpu().numpy(), want[q]), "mixed", infm[q],
              rel(xm[q].cpu().numpy(), want[q]), flush=True)
        assert inf[q]["status"] == 0 and rel(x[q].cpu().numpy(), want[q]) < 1e-10
        assert infm[q]["status"] == 0 and infm[q]["rel_res_true"] <= 1e-7
        assert rel(xm[q].cpu().numpy(), want[q]) < 1e-5
    # transposed system A^T y = b with M^T
    wt = solve.solve_dense(A.T, b[1])
    y, inft = ctx.solve_T(bt[1], i_omega=1, tol=1e-12, maxit=1000, precision="c128")
    ym, inftm = ctx.solve_T(bt[1], i_omega=1, tol=1e-7, maxit=1000, precision="mixed")
    print("transposed", inft, rel(y.cpu().numpy(), wt), inftm, rel(ym.cpu().numpy(), wt), flush=True)
    assert rel(y.cpu().numpy(), wt) < 1e-10 and rel(ym.cpu().numpy(), wt) < 1e-5
    # warm start from the solution: converged at once
    x0, inf0 = ctx.solve(bt[:1], i_omega=1, tol=1e-10, precision="c128", x0=x[:1].clone())
    assert inf0[0]["iters"] <= 1 and rel(x0[0].cpu().numpy(), want[0]) < 1e-10
    ctx.close()


def test_multi_frequency_preconditioned_solve_equals_solo_solves():
    m = medium((10, 9, 8), 35, rel_=0.25, background="vti")
    ctx = lsvie.context_from_model(m, omegas=WS, precision="mixed", max_rhs=4, precond="block_jacobi")
    freqs = [1, 0, 1, 0]
    srcs = [(4, 4, 3), (2, 5, 6), (8, 1, 2), (5, 5, 5)]
    b = torch.stack([ctx.rhs_moment(np.eye(6)[q], s, i_omega=iw) for q, (iw, s) in enumerate(zip(freqs, srcs))])
    for precision, tol in (("c128", 1e-11), ("mixed", 1e-7)):
        x, infos = ctx.solve(b, i_omega=freqs, tol=tol, maxit=2000, precision=precision)
        for q, iw in enumerate(freqs):
            xq, iq = ctx.solve(b[q], i_omega=iw, tol=tol, maxit=2000, precision=precision)
            assert torch.equal(x[q], xq), (precision, q)
            assert infos[q]["iters"] == iq[0]["iters"] and infos[q]["status"] == 0
        print(precision, [i["iters"] for i in infos], flush=True)
    P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, WS[0])
    want = solve.solve_dense(P.dense_A(), b[1].cpu().numpy())
    assert rel(x[1].cpu().numpy(), want) < 1e-5
    ctx.close()


def test_fewer_matvecs_on_strong_contrast():
    """16^3, +-35 % random contrast at 40 Hz: the preconditioned solve needs clearly fewer matvecs and
    reaches the same field."""
    m = models.random_medium((16, 16, 16), 5, rel=0.35, h=10.0, aniso_background=True)
    w = [2 * np.pi * 40.0]
    plain = lsvie.context_from_model(m, omegas=w, precision="mixed")
    pre = lsvie.context_from_model(m, omegas=w, precision="mixed", precond="block_jacobi")
    b = plain.rhs_moment(np.eye(6)[0], (8, 8, 8))
    for precision, tol in (("c128", 1e-8), ("mixed", 1e-6)):
        x0, i0 = plain.solve(b, tol=tol, maxit=4000, precision=precision)
        x1, i1 = pre.solve(b, tol=tol, maxit=4000, precision=precision)
        print(precision, "matvecs plain", i0[0]["matvecs"], "block Jacobi", i1[0]["matvecs"], flush=True)
        assert i0[0]["status"] == 0 and i1[0]["status"] == 0
        assert i1[0]["matvecs"] < 0.85 * i0[0]["matvecs"]
        assert rel(x1.cpu().numpy(), x0.cpu().numpy()) < 10 * tol
    plain.close()
    pre.close()


@pytest.mark.parametrize("which", ["config3", "config5"])
def test_sampled_blocks_at_128(which):
    """The 128^3 grids of the benchmark (closed-form table, VTI folded) and of the uneven batch (anisotropic
    octant table): inverse blocks at 40 sampled cells (corners and faces included) against the oracle's
    per-cell construction."""
    if which == "config3":
        m = models.config3(n=128, freqs=(40.0,))
        mode, bar = "exact", 1e-12
    else:
        m = models.config5(n=128, freqs=(50.0,))
        mode, bar = "aniso", 1e-9
    ctx = lsvie.context_from_model(m, precision="mixed", green_mode=mode, precond="block_jacobi")
    got = ctx.precond_blocks(0).cpu().numpy()
    ctx.close()
    rng = np.random.default_rng(7)
    cells = np.concatenate([np.array([[0, 0, 0], [127, 127, 127], [0, 127, 64], [127, 1, 0], [64, 64, 127]]),
                            rng.integers(0, 128, size=(35, 3))])
    P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, m.omegas[0], mode=mode)
    D = precond.block_diagonal_at(P, cells)
    g = got[cells[:, 2], cells[:, 1], cells[:, 0]]
    e = block_err(g, D)
    print(which, "sampled inverse blocks vs oracle", e, "max |D - I|", np.abs(D - np.eye(3)).max(), flush=True)
    assert e < bar
