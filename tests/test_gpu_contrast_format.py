"""The orthotropic contrast format: for media whose total contrast vanishes off the entries 11, 12, 13, 22, 23,
33, 44, 55, 66 at every cell (isotropic and VTI here), the fused contrast kernel reads 9 values per cell instead
of 21 and treats the rest as exact zeros (Eq 8, 11-12).  Its operator must equal the general kernel's value for
value (the products it drops are exact zeros), forward and transposed, in both precisions, and it must match
the oracle; a general-anisotropic medium keeps 21 values."""

import numpy as np
import pytest

from oracle import operator as op
from paper_2301_12836_amd import models

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2301_12836_amd import lsvie  # noqa: E402


def context(m, w, general, monkeypatch):
    if general:
        monkeypatch.setenv("LS_CONTRAST_K", "21")
    else:
        monkeypatch.delenv("LS_CONTRAST_K", raising=False)
    return lsvie.context_from_model(m, omegas=[w], precision="mixed", max_rhs=2)


@pytest.mark.parametrize("which", ["iso", "vti"])
def test_orthotropic_format_equals_general(which, monkeypatch):
    m = models.config1() if which == "iso" else models.config2(n=24)
    w = m.omegas[0]
    auto = context(m, w, False, monkeypatch)
    gen = context(m, w, True, monkeypatch)
    assert auto.contrast_format == 9 and gen.contrast_format == 21
    u = torch.from_numpy(np.stack([models.random_field(m.shape, seed=s) for s in (3, 4)]))
    for dt in (torch.complex128, torch.complex64):
        uu = u.to(dt)
        a, g = auto.apply(uu), gen.apply(uu)
        assert torch.equal(a, g), f"{which} {dt} forward"
    assert torch.equal(auto.apply_T(u), gen.apply_T(u)), f"{which} transposed"
    # the FP32 transposed operator inside a mixed transposed solve: fixed-order reductions, so equal operators
    # give equal iterates
    xa, ia = auto.solve_T(u, tol=1e-6, maxit=500, precision="mixed")
    xg, ig = gen.solve_T(u, tol=1e-6, maxit=500, precision="mixed")
    assert torch.equal(xa, xg) and [i["iters"] for i in ia] == [i["iters"] for i in ig], f"{which} mixed solve_T"
    P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, w)
    got = auto.apply(u).cpu().numpy()
    for r in range(2):
        want = P.apply_fft(u[r].numpy())
        e = np.linalg.norm(got[r] - want) / np.linalg.norm(want)
        print(which, "rhs", r, "c128 vs oracle", e, flush=True)
        assert e < 1e-10
    auto.close()
    gen.close()


def test_general_medium_keeps_21_values(monkeypatch):
    m = models.random_medium((12, 10, 8), seed=5, rel=0.1)
    ctx = context(m, 2 * np.pi * 15.0, False, monkeypatch)
    assert ctx.contrast_format == 21
    ctx.close()


def test_set_contrast_switches_format(monkeypatch):
    """A context built on an isotropic medium (9 values per cell) given a general contrast by ls_set_contrast
    switches to 21 and applies exactly the operator of a context built on that contrast; and back."""
    m = models.config1(n=12)
    w = m.omegas[0]
    g = models.random_medium(m.shape, seed=8, rel=0.1)
    ctx = context(m, w, False, monkeypatch)
    assert ctx.contrast_format == 9
    ctx.set_contrast(g.dc21, g.drho)
    assert ctx.contrast_format == 21
    fresh = lsvie.Context(m.shape, m.h, m.C0, m.rho0, g.dc21, g.drho, [w], precision="mixed", max_rhs=2)
    u = torch.from_numpy(np.stack([models.random_field(m.shape, seed=s) for s in (1, 2)]))
    for dt in (torch.complex128, torch.complex64):
        assert torch.equal(ctx.apply(u.to(dt)), fresh.apply(u.to(dt)))
    ctx.set_contrast(m.dc21, m.drho)
    assert ctx.contrast_format == 9
    back = context(m, w, False, monkeypatch)
    assert torch.equal(ctx.apply(u), back.apply(u))
    for c in (ctx, fresh, back):
        c.close()
