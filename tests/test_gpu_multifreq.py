"""Systems at different frequencies in one solve: ls_solve_multi and ls_solve_batch put every system of a
context into the same operator launches and Bi-CGSTAB kernels, each at its own frequency (its own
Green's table and w^2), with converged systems dropping out of the launches.  Every decision is taken per
system, so each result must be bitwise the one the system's solo solve returns; the FP64 results are
also held to the oracle's dense LU solution."""

import numpy as np
import pytest

from oracle import operator as op, solve
from paper_2301_12836_amd import models

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2301_12836_amd import lsvie  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


FREQS = [9.0, 21.0, 33.0]
SYSTEMS = [(2, np.eye(6)[0], (5, 4, 4)), (0, models.EXPLOSION, (3, 5, 2)), (1, models.double_couple(30, 60, 90), (6, 4, 5)),
           (0, np.eye(6)[4], (0, 9, 8)), (2, models.double_couple(0, 90, 0), (11, 0, 3)), (1, np.eye(6)[2], (5, 4, 4))]


@pytest.mark.parametrize("precision,tol,width", [("c128", 1e-12, "0"), ("mixed", 1e-7, "0"), ("mixed", 1e-7, "2")])
def test_solve_multi_equals_solo_solves_and_dense(precision, tol, width, monkeypatch):
    """width: the most systems one operator launch covers (LS_LAUNCH_RHS; 0 no cap, 2 splits every launch)."""
    monkeypatch.setenv("LS_LAUNCH_RHS", width)
    m = models.random_medium((12, 10, 9), seed=41, rel=0.12, aniso_background=True)
    ws = [2 * np.pi * f for f in FREQS]
    ctx = lsvie.context_from_model(m, omegas=ws, precision="mixed", max_rhs=6)
    freqs = [s[0] for s in SYSTEMS]
    b = torch.stack([ctx.rhs_moment(M, src, i_omega=iw) for iw, M, src in SYSTEMS])
    x, infos = ctx.solve(b, i_omega=freqs, tol=tol, maxit=2000, precision=precision)
    for q, (iw, M, src) in enumerate(SYSTEMS):
        xq, iq = ctx.solve(b[q], i_omega=iw, tol=tol, maxit=2000, precision=precision)
        print(precision, "system", q, "freq", FREQS[iw], infos[q], flush=True)
        assert torch.equal(x[q], xq), f"system {q} differs from its solo solve"
        for k in ("iters", "matvecs", "refinements", "status"):
            assert infos[q][k] == iq[0][k], (q, k, infos[q][k], iq[0][k])
        assert infos[q]["status"] == 0 and infos[q]["rel_res_true"] <= tol
    # the systems need different iteration counts, so some left the launches before others
    assert len({i["iters"] for i in infos}) > 1
    for q in (0, 1, 2):
        iw, M, src = SYSTEMS[q]
        P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, ws[iw])
        want = solve.solve_dense(P.dense_A(), P.rhs_moment(M, src))
        e = rel(x[q].cpu().numpy(), want)
        print(precision, "system", q, "vs dense", e, flush=True)
        assert e < (1e-10 if precision == "c128" else 1e-5)
    ctx.close()


def test_one_batch_call_over_frequencies_equals_per_frequency_solves():
    """The benchmark's form at 16^3: 6 elementary moment tensors x 4 frequencies as 24 jobs in one
    ls_solve_batch call on one context (one mixed-frequency solve), against one 6-system ls_solve per
    frequency: bitwise equal fields and equal iteration and matvec counts."""
    m = models.config3(n=16, h=16.0, freqs=(5, 15, 25, 40))
    ctx = lsvie.context_from_model(m, precision="mixed", max_rhs=24)
    jobs = [(0, iw, M, src, 0.0) for iw in range(4) for M, src in m.sources]
    outs, infos = lsvie.solve_batch([ctx], jobs, tol=1e-6, maxit=2000, precision="mixed")
    for iw in range(4):
        b = torch.stack([ctx.rhs_moment(M, src, i_omega=iw) for M, src in m.sources])
        x, inf = ctx.solve(b, i_omega=iw, tol=1e-6, maxit=2000, precision="mixed")
        for J in range(6):
            k = 6 * iw + J
            assert torch.equal(outs[k], x[J]), (iw, J)
            assert infos[k]["iters"] == inf[J]["iters"] and infos[k]["matvecs"] == inf[J]["matvecs"]
            assert infos[k]["status"] == 0 and infos[k]["rel_res_true"] <= 1e-6
        print("freq", m.freqs[iw], "iterations", [i["iters"] for i in inf], flush=True)
    ctx.close()
