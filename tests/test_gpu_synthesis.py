"""GPU parity of the time-domain synthesis: receiver sampling, the inverse transform with the Ricker
wavelet against the oracle's, and whole seismograms of a small heterogeneous model against the oracle's
per-frequency dense solves."""

import numpy as np
import pytest

from oracle import operator as op, solve, synthesis as osyn
from paper_2301_12836_amd import models

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2301_12836_amd import lsvie, synthesis  # noqa: E402


def test_sample_and_synthesize_match_oracle():
    m = models.random_medium((8, 7, 6), seed=1)
    ctx = lsvie.context_from_model(m, omegas=[2 * np.pi * 10.0])
    u = torch.from_numpy(np.stack([models.random_field(m.shape, s) for s in range(2)])).to(ctx.device)
    rec = np.array([[0, 0, 0], [7, 6, 5], [3, 2, 4]])
    got = ctx.sample(u, rec).cpu().numpy()
    un = u.cpu().numpy()
    assert np.array_equal(got, np.transpose(un[:, :, rec[:, 2], rec[:, 1], rec[:, 0]], (0, 2, 1)))
    rng = np.random.default_rng(3)
    nt, dt = 96, 0.002
    k = np.array([0, 1, 2, 5, 17, 30, 48])           # includes zero and Nyquist
    U = rng.normal(size=(len(k), 5)) + 1j * rng.normal(size=(len(k), 5))
    w = 2 * np.pi * k / (nt * dt)
    for fp, ts in ((25.0, 0.05), (0.0, 0.0)):
        S = osyn.ricker_spectrum(w, fp, ts) if fp > 0 else np.ones(len(k))
        want = osyn.traces(S[:, None] * U, k, nt, dt)
        tr = ctx.synthesize(torch.from_numpy(U), k, nt, dt, fp, ts).cpu().numpy()
        assert np.abs(tr - want).max() <= 1e-12 * np.abs(want).max()
    with pytest.raises(lsvie.LsError):
        ctx.synthesize(torch.from_numpy(U), np.array([0, 1, 2, 5, 17, 30, 49]), nt, dt)
    with pytest.raises(lsvie.LsError):
        ctx.sample(u, np.array([[8, 0, 0]]))
    ctx.close()


def test_seismograms_match_oracle_dense_solves():
    """10^3 heterogeneous model, explosion and double couple, 4 receivers, Ricker 25 Hz: the library's
    frequency loop, batched solves, sampling and synthesis against dense oracle solves per frequency."""
    m = models.random_medium((10, 10, 10), seed=5, rel=0.1, aniso_background=True)
    sources = [(models.EXPLOSION, (5, 5, 4), 0.0), (models.double_couple(30, 60, 90), (3, 6, 5), 0.01)]
    rec = np.array([[0, 0, 0], [9, 2, 0], [5, 9, 9], [2, 5, 7]])
    nt, dt, fp, ts = 128, 0.002, 25.0, 0.06
    traces, k, infos = synthesis.seismograms(m, sources, rec, nt, dt, fp, ts, eps=1e-4, tol=1e-11,
                                             precision="c128", chunk=8)
    assert all(i["status"] == 0 for i in infos)
    assert np.array_equal(k, osyn.synthesis_indices(nt, dt, fp, 1e-4))
    U = np.zeros((len(k), len(sources), len(rec), 3), dtype=complex)
    for q, kk in enumerate(k):
        w = 2 * np.pi * kk / (nt * dt)
        P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, w)
        A = P.dense_A()
        for s, (M, src, t0) in enumerate(sources):
            u = solve.solve_dense(A, P.rhs_moment(M, src, t0))
            U[q, s] = u[:, rec[:, 2], rec[:, 1], rec[:, 0]].T
    S = osyn.ricker_spectrum(2 * np.pi * k / (nt * dt), fp, ts)
    want = osyn.traces(S[:, None, None, None] * U, k, nt, dt)
    got = traces.cpu().numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    print("frequencies", len(k), "max relative trace error", err, flush=True)
    assert err < 1e-8


def test_seismograms_with_the_anisotropic_background_tensor():
    """The same pipeline with the VTI background as its own Green's tensor (LS_GREEN_ANISO) and BiCGSTAB(2),
    on a 6^3 model, against dense oracle solves with the oracle's anisotropic tensor."""
    m = models.random_medium((6, 6, 6), seed=9, rel=0.1, aniso_background=True)
    sources = [(models.double_couple(30, 60, 90), (3, 2, 3), 0.0)]
    rec = np.array([[0, 0, 0], [5, 1, 0], [2, 5, 5]])
    nt, dt, fp, ts = 64, 0.004, 15.0, 0.08
    traces, k, infos = synthesis.seismograms(m, sources, rec, nt, dt, fp, ts, eps=1e-3, tol=1e-11,
                                             precision="c128", chunk=8, green_mode="aniso", bicgstab_l=2)
    assert all(i["status"] == 0 for i in infos)
    U = np.zeros((len(k), len(sources), len(rec), 3), dtype=complex)
    for q, kk in enumerate(k):
        w = 2 * np.pi * kk / (nt * dt)
        P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, w, mode="aniso")
        A = P.dense_A()
        for s, (M, src, t0) in enumerate(sources):
            u = solve.solve_dense(A, P.rhs_moment(M, src, t0))
            U[q, s] = u[:, rec[:, 2], rec[:, 1], rec[:, 0]].T
    S = osyn.ricker_spectrum(2 * np.pi * k / (nt * dt), fp, ts)
    want = osyn.traces(S[:, None, None, None] * U, k, nt, dt)
    err = np.abs(traces.cpu().numpy() - want).max() / np.abs(want).max()
    print("anisotropic background: frequencies", len(k), "max relative trace error", err, flush=True)
    assert err < 1e-8
