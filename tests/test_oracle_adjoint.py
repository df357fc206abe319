"""Pins of the oracle's transposed operator and dense-adjoint misfit gradient.

The transposed apply is checked against the transpose of the dense matrix; the gradient for the
contrast, the density contrast and the moment tensor against central finite differences of the misfit
computed with dense LU solves (an independent route through the same definitions).
"""

import numpy as np
import pytest

from oracle import adjoint, operator as op
from paper_2301_12836_amd import models

H = 10.0


def setup_case(seed=3):
    shape = (4, 5, 4)
    m = models.random_medium(shape, seed, rel=0.1, h=H, aniso_background=True)
    omegas = [2 * np.pi * 12.0, 2 * np.pi * 19.0]
    probs = [op.Problem(shape, H, m.C0, m.rho0, m.dc21, m.drho, w) for w in omegas]
    sources = [(models.double_couple(30, 60, 90), (1, 2, 1), 0.0), (models.EXPLOSION, (2, 3, 2), 0.004)]
    receivers = np.array([[0, 0, 0], [3, 4, 0], [1, 2, 3]])
    rng = np.random.default_rng(seed)
    data = [[rng.normal(size=(3, 3)) * 1e-15 + 1j * rng.normal(size=(3, 3)) * 1e-15 for _ in sources]
            for _ in omegas]
    return m, omegas, probs, sources, receivers, data


def test_apply_T_is_dense_transpose():
    m, omegas, probs, *_ = setup_case()
    P = probs[0]
    y = models.random_field(m.shape, 4)
    want = (P.dense_A().T @ y.ravel()).reshape(y.shape)
    assert np.abs(adjoint.apply_T(P, y) - want).max() < 1e-13 * np.abs(want).max()


def _J(m, omegas, sources, receivers, data, dc21=None, drho=None, Ms=None):
    dc = m.dc21 if dc21 is None else dc21
    dr = m.drho if drho is None else drho
    probs = [op.Problem(m.shape, H, m.C0, m.rho0, dc, dr, w) for w in omegas]
    srcs = sources if Ms is None else [(M, s, t0) for M, (_, s, t0) in zip(Ms, sources)]
    return adjoint.misfit(probs, srcs, receivers, data)[0]


@pytest.mark.slow
def test_gradient_matches_central_differences():
    m, omegas, probs, sources, receivers, data = setup_case()
    J, g21, grho, gM = adjoint.misfit_gradient_dense(probs, sources, receivers, data)
    assert np.isclose(J, _J(m, omegas, sources, receivers, data), rtol=1e-12)
    checks = 0
    for (q, cell) in [(0, (1, 2, 1)), (4, (2, 1, 3)), (15, (0, 4, 2)), (20, (3, 3, 0)), (7, (1, 2, 2))]:
        i, j, k = cell
        d = 1e5
        dp = m.dc21.copy(); dp[q, k, j, i] += d
        dm = m.dc21.copy(); dm[q, k, j, i] -= d
        fd = (_J(m, omegas, sources, receivers, data, dc21=dp) - _J(m, omegas, sources, receivers, data, dc21=dm)) / (2 * d)
        assert abs(fd - g21[q, k, j, i]) <= 1e-5 * abs(fd) + 1e-12 * np.abs(g21).max(), (q, cell)
        checks += 1
    i, j, k = (2, 3, 1)
    d = 1e-2
    rp = m.drho.copy(); rp[k, j, i] += d
    rm = m.drho.copy(); rm[k, j, i] -= d
    fd = (_J(m, omegas, sources, receivers, data, drho=rp) - _J(m, omegas, sources, receivers, data, drho=rm)) / (2 * d)
    assert abs(fd - grho[k, j, i]) <= 1e-5 * abs(fd)
    for isrc in range(2):
        for J_ in (0, 3, 5):
            d = 1e-4
            Mp = [np.array(s[0], dtype=float) for s in sources]
            Mm = [np.array(s[0], dtype=float) for s in sources]
            Mp[isrc][J_] += d
            Mm[isrc][J_] -= d
            fd = (_J(m, omegas, sources, receivers, data, Ms=Mp) - _J(m, omegas, sources, receivers, data, Ms=Mm)) / (2 * d)
            assert abs(fd - gM[isrc, J_]) <= 1e-6 * abs(fd) + 1e-9 * np.abs(gM).max()


def test_vti_chain_rule_matches_direct_differences():
    m, omegas, probs, sources, receivers, data = setup_case(5)
    J, g21, grho, gM = adjoint.misfit_gradient_dense(probs, sources, receivers, data)
    gv = adjoint.vti_chain(g21)
    # perturb C66 at one cell through the VTI relations: C66 += d and C12 -= 2 d
    i, j, k = (1, 1, 1)
    d = 1e5
    idx = {pair: n for n, pair in enumerate(op.UPPER21)}
    dp = m.dc21.copy(); dp[idx[(5, 5)], k, j, i] += d; dp[idx[(0, 1)], k, j, i] -= 2 * d
    dm = m.dc21.copy(); dm[idx[(5, 5)], k, j, i] -= d; dm[idx[(0, 1)], k, j, i] += 2 * d
    fd = (_J(m, omegas, sources, receivers, data, dc21=dp) - _J(m, omegas, sources, receivers, data, dc21=dm)) / (2 * d)
    assert abs(fd - gv[3, k, j, i]) <= 1e-5 * abs(fd)
