"""The allocation-free apply (ls_apply_noalloc, for callers that cannot allocate device memory) against
ls_apply through the C ABI: bitwise equal outputs on two calls in a row, the second on a smaller input
(so the shared scratch array still holds the first call's larger contents), the oracle's apply on both, and
the size limit of the scratch array."""

import numpy as np
import pytest

from oracle import operator as op
from paper_2301_12836_amd import models

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2301_12836_amd import lsvie  # noqa: E402

W = 2 * np.pi * 17.0


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def both_applies(ctx, u):
    """(ls_apply, ls_apply_noalloc) outputs of the fields u [n_rhs, 3, N3, N2, N1] through the C ABI."""
    nrhs = u.shape[0]
    a = torch.empty_like(u)
    b = torch.full_like(u, complex(np.nan, np.nan))
    lsvie.ls_apply(ctx.handle, 0, u, a, nrhs)
    lsvie.ls_apply_noalloc(ctx.handle, 0, u, b, nrhs)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_noalloc_apply_equals_apply_on_two_calls_larger_then_smaller():
    cases = [((24, 20, 18), 2, 31), ((12, 10, 9), 1, 32)]   # the second input is smaller than the first
    for shape, nrhs, seed in cases:
        m = models.random_medium(shape, seed=seed, rel=0.1, aniso_background=True)
        ctx = lsvie.context_from_model(m, omegas=[W], max_rhs=2)
        un = np.stack([models.random_field(shape, seed=seed + r) for r in range(nrhs)])
        u = torch.from_numpy(un).to(ctx.device)
        want, got = both_applies(ctx, u)
        print(shape, nrhs, "bitwise equal", np.array_equal(got, want), flush=True)
        assert np.array_equal(got, want)
        P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, W)
        for r in range(nrhs):
            e = rel(got[r], P.apply_fft(un[r]))
            print(shape, "rhs", r, "vs oracle", e, flush=True)
            assert e < 1e-10
        ctx.close()


def test_noalloc_apply_size_limit():
    """One 64^3 field needs 3 x 64 x 128 x 128 x 16 = 50 MB of work buffer (fits the 64 MiB array); two
    need 100 MB and are refused before any launch."""
    shape = (64, 64, 64)
    m = models.random_medium(shape, seed=5, rel=0.1)
    ctx = lsvie.context_from_model(m, omegas=[W], max_rhs=2)
    u = torch.from_numpy(np.stack([models.random_field(shape, seed=s) for s in (1, 2)])).to(ctx.device)
    want, got = both_applies(ctx, u[:1].contiguous())
    assert np.array_equal(got, want)
    out = torch.empty_like(u)
    with pytest.raises(lsvie.LsError) as e:
        lsvie.ls_apply_noalloc(ctx.handle, 0, u, out, 2)
    assert e.value.code == lsvie.LS_ERR_ARG
    ctx.close()
