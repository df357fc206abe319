"""GPU BiCGSTAB(l) (ls_options.bicgstab_l > 1) against the oracle: the dense LU solution, the oracle's
BiCGSTAB(l) residual history (same method, its published modified Gram-Schmidt form against the
library's Gram-matrix form: equal iterates in exact arithmetic), batch invariance, and the status
codes of the failure paths."""

import numpy as np
import pytest

from oracle import operator as op, solve
from paper_2301_12836_amd import models

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2301_12836_amd import lsvie  # noqa: E402

W15 = 2 * np.pi * 15.0


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def to_np(t):
    return t.detach().cpu().numpy()


def hard_problem():
    m = models.random_medium((6, 5, 7), seed=31, rel=0.3)
    return m, op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, W15)


@pytest.mark.parametrize("ell", [2, 3, 4])
def test_solution_matches_dense_oracle(ell):
    m, P = hard_problem()
    b = P.rhs_moment(models.EXPLOSION, (2, 2, 3))
    want = solve.solve_dense(P.dense_A(), b)
    ctx = lsvie.context_from_model(m, omegas=[W15], precision="mixed", bicgstab_l=ell)
    bg = torch.from_numpy(b).to(ctx.device)
    u, info = ctx.solve(bg, tol=1e-12, maxit=400, precision="c128")
    print("l", ell, "c128", rel(to_np(u), want), info, flush=True)
    assert info[0]["status"] == 0 and info[0]["rel_res_true"] <= 1e-12
    assert rel(to_np(u), want) < 1e-10
    assert info[0]["matvecs"] <= 2 * info[0]["iters"] + 1
    u, info = ctx.solve(bg, tol=1e-7, maxit=400, precision="mixed")
    print("l", ell, "mixed", rel(to_np(u), want), info, flush=True)
    assert info[0]["status"] == 0 and rel(to_np(u), want) < 1e-5
    ctx.close()


def test_residual_history_matches_oracle_bicgstab_l():
    m, P = hard_problem()
    b = P.rhs_moment(models.EXPLOSION, (2, 2, 3))
    ctx = lsvie.context_from_model(m, omegas=[W15], bicgstab_l=4)
    u, info = ctx.solve(torch.from_numpy(b).to(ctx.device), tol=1e-11, maxit=400)
    h = ctx.residual_history(0)
    _, hist, nmv = solve.bicgstab_l(P.apply_fft, b, 1e-11, 4)
    print("steps", len(h), len(hist) - 1, "first", h[:5], hist[1:6], flush=True)
    assert len(h) == info[0]["iters"] and abs(len(h) - (len(hist) - 1)) <= 4
    for i in range(8):
        assert abs(h[i] - hist[i + 1]) <= 1e-6 * hist[i + 1]
    ctx.close()


def test_batched_solve_is_bitwise_equal_to_single():
    m, P = hard_problem()
    ctx = lsvie.context_from_model(m, omegas=[W15], max_rhs=3, bicgstab_l=4)
    srcs = [(models.EXPLOSION, (2, 2, 3)), (models.double_couple(30, 60, 90), (3, 1, 4)),
            (np.eye(6)[4], (1, 3, 2))]
    bs = torch.stack([ctx.rhs_moment(M, s) for M, s in srcs])
    U, infos = ctx.solve(bs, tol=1e-10, maxit=400)
    for k in range(3):
        u, info = ctx.solve(bs[k], tol=1e-10, maxit=400)
        assert torch.equal(U[k], u), k
        assert info[0]["iters"] == infos[k]["iters"]
    ctx.close()


def test_initial_guess_and_failure_codes():
    m, P = hard_problem()
    ctx = lsvie.context_from_model(m, omegas=[W15], precision="mixed", bicgstab_l=2)
    b = ctx.rhs_moment(models.EXPLOSION, (2, 2, 3))
    u, _ = ctx.solve(b, tol=1e-11, maxit=400, precision="c128")
    # a converged initial guess: A x0 and the true residual (c128), the true residual only (mixed)
    _, info = ctx.solve(b, tol=1e-9, maxit=400, x0=u, precision="c128")
    assert info[0]["status"] == 0 and info[0]["iters"] == 0 and info[0]["matvecs"] == 2
    _, info = ctx.solve(b, tol=1e-9, maxit=400, x0=u, precision="mixed")
    assert info[0]["status"] == 0 and info[0]["iters"] == 0 and info[0]["matvecs"] == 1
    _, info = ctx.solve(b, tol=1e-14, maxit=4, precision="c128", raise_on_error=False)
    assert info[0]["status"] == lsvie.LS_ERR_NOT_CONVERGED and info[0]["iters"] <= 4
    ctx.close()
    dc = m.dc21.copy()
    dc[0, 3, 3, 3] = np.nan
    ctx = lsvie.Context(m.shape, m.h, m.C0, m.rho0, dc, m.drho, [W15], precision="mixed", bicgstab_l=4)
    for prec in ("c128", "mixed"):
        _, infos = ctx.solve(b, tol=1e-8, precision=prec, raise_on_error=False)
        assert infos[0]["status"] == lsvie.LS_ERR_NONFINITE, (prec, infos)
    ctx.close()
    with pytest.raises(lsvie.LsError):
        lsvie.context_from_model(m, omegas=[W15], bicgstab_l=5)


@pytest.mark.parametrize("ell", [1, 4])
def test_unconverged_solve_returns_its_best_iterate(ell):
    """A solve stopped by maxit returns the iterate with (within a factor 2) the smallest residual seen,
    never a worse last iterate: the saved copy is refreshed whenever the residual halves."""
    m, P = hard_problem()
    ctx = lsvie.context_from_model(m, omegas=[W15], bicgstab_l=ell)
    b = ctx.rhs_moment(models.EXPLOSION, (2, 2, 3))
    for maxit in (4, 8, 12):   # whole BiCGSTAB(4) cycles
        u, info = ctx.solve(b, tol=1e-14, maxit=maxit, precision="c128", raise_on_error=False)
        h = np.array(ctx.residual_history(0))
        assert info[0]["status"] == lsvie.LS_ERR_NOT_CONVERGED
        true = info[0]["rel_res_true"]
        print("l", ell, "maxit", maxit, "history", h, "returned", true, flush=True)
        assert true <= 2.0 * (1 + 1e-6) * min(h.min(), 1.0)
        assert true <= h[-1] * (1 + 1e-6)
    ctx.close()


def test_transposed_solve_and_uneven_batch_with_bicgstab_l():
    """BiCGSTAB(4) behind the adjoint solve (A^T, no fused inner products) matches the dense transpose
    solve, and a batch over two contexts with different grids and l matches each job's single solve."""
    m, P = hard_problem()
    ctx = lsvie.context_from_model(m, omegas=[W15], precision="mixed", bicgstab_l=4)
    b = models.random_field(m.shape, 3)
    want = solve.solve_dense(P.dense_A().T, b)
    x, info = ctx.solve_T(torch.from_numpy(b), tol=1e-12, maxit=600, precision="c128")
    print("solve_T l=4", rel(to_np(x), want), info, flush=True)
    assert rel(to_np(x), want) < 1e-10
    xm, info = ctx.solve_T(torch.from_numpy(b), tol=1e-7, maxit=600, precision="mixed")
    assert rel(to_np(xm), want) < 1e-5
    mb = models.random_medium((9, 7, 8), seed=8, rel=0.2, aniso_background=True)
    B = lsvie.context_from_model(mb, omegas=[W15], precision="mixed", max_rhs=2, bicgstab_l=2)
    jobs = [(0, 0, models.EXPLOSION, (2, 2, 3), 0.0), (1, 0, models.double_couple(30, 60, 90), (4, 3, 4), 0.0),
            (1, 0, np.eye(6)[2], (1, 5, 6), 0.001)]
    outs, infos = lsvie.solve_batch([ctx, B], jobs, tol=1e-10, maxit=600, precision="c128")
    for (ci, iw, M, src, t0), u, inf in zip(jobs, outs, infos):
        c = (ctx, B)[ci]
        single, _ = c.solve(c.rhs_moment(M, src, i_omega=iw, t0=t0), i_omega=iw, tol=1e-10, maxit=600,
                            precision="c128")
        assert inf["status"] == 0 and rel(to_np(u), to_np(single)) < 1e-9, (ci, src)
    ctx.close()
    B.close()
