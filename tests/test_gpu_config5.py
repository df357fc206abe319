"""The large uneven configuration at its full sizes: 256^3 (h 6 m), 192^3 (h 8 m) and 128^3 (h 12 m) grids
over an orthorhombic background with layered plus random-field contrast.  The operator is checked against
the oracle's direct sums at sampled cells (the oracle cannot form a whole 256^3 field in seconds); the
mixed-precision batched solve over the three grids is checked by its FP64 true residual."""

import numpy as np
import pytest

from oracle import operator as op
from paper_2301_12836_amd import models

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2301_12836_amd import lsvie  # noqa: E402

_MODELS = {}


def model(n):
    if n not in _MODELS:
        _MODELS[n] = models.config5(n)
    return _MODELS[n]


@pytest.mark.parametrize("n,cells", [(256, [(128, 128, 128), (0, 255, 3)]), (192, [(5, 100, 191)])])
def test_config5_apply_sampled_cells(n, cells):
    m = model(n)
    w = m.omegas[-1]  # 50 Hz, the shortest wavelength
    ctx = lsvie.context_from_model(m, omegas=[w], precision="mixed")
    u = models.random_field(m.shape, 5)
    ut = torch.from_numpy(u).to(ctx.device)
    got = ctx.apply(ut)
    got32 = ctx.apply(ut.to(torch.complex64))
    cells = np.array(cells)
    g = got[:, cells[:, 2], cells[:, 1], cells[:, 0]].T.cpu().numpy()
    g32 = got32[:, cells[:, 2], cells[:, 1], cells[:, 0]].T.cpu().numpy()
    ctx.close()
    del got, got32, ut
    P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, w)
    want = P.apply_bruteforce(u, cells)
    for t in range(len(cells)):
        e = np.linalg.norm(g[t] - want[t]) / np.linalg.norm(want[t])
        e32 = np.linalg.norm(g32[t] - want[t]) / np.linalg.norm(want[t])
        print(n, cells[t], "c128", e, "c64", e32, flush=True)
        assert e < 1e-10 and e32 < 1e-5


def test_config5_batched_solve_over_the_three_grids():
    """One job per grid (an elementary moment tensor at the centre, 10 Hz) in one ls_solve_batch call,
    mixed precision to 1e-6; each context's FP64 true residual certifies its solution."""
    ctxs = [lsvie.context_from_model(model(n), omegas=model(n).omegas[:1], precision="mixed")
            for n, _ in models.CONFIG5_GRIDS]
    jobs = [(i, 0, np.eye(6)[(2 * i) % 6], (n // 2,) * 3, 0.0) for i, (n, _) in enumerate(models.CONFIG5_GRIDS)]
    outs, infos = lsvie.solve_batch(ctxs, jobs, tol=1e-6, maxit=3000, precision="mixed")
    for (n, _), u, info, ctx in zip(models.CONFIG5_GRIDS, outs, infos, ctxs):
        print(n, info, flush=True)
        assert info["status"] == 0 and info["rel_res_true"] <= 1e-6
        assert bool(torch.isfinite(u).all()) and float(u.abs().max()) > 0
        ctx.close()
