"""GPU tests of the batching machinery: graph-captured BiCGSTAB iterations (bitwise equal to eager
launches, repeated solves re-capturing), autotuned FFT kernel variants (parity with the oracle), and
the explicit LDS Stockham variant against the register four-step variant."""

import numpy as np
import pytest

from oracle import operator as op
from paper_2301_12836_amd import models

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2301_12836_amd import lsvie  # noqa: E402

W = 2 * np.pi * 17.0


def rel(a, b):
    return np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel())


@pytest.mark.parametrize("precision", ["c128", "mixed"])
def test_graph_iterations_equal_eager_launches(precision):
    m = models.random_medium((20, 18, 16), seed=6, rel=0.1, aniso_background=True)
    eager = lsvie.context_from_model(m, omegas=[W], precision="mixed", max_rhs=3, graphs=False)
    graph = lsvie.context_from_model(m, omegas=[W], precision="mixed", max_rhs=3, graphs=True)
    src = (9, 8, 7)
    b = torch.stack([eager.rhs_moment(np.eye(6)[J], src) for J in (0, 3, 5)])
    x_e, inf_e = eager.solve(b, tol=1e-9, precision=precision)
    for rep in range(3):   # each solve captures and replays its own graph; eager work in between
        x_g, inf_g = graph.solve(b, tol=1e-9, precision=precision)
        _ = graph.apply(b)
        assert torch.equal(x_g, x_e), f"replay {rep} differs from eager launches"
        assert [i["iters"] for i in inf_g] == [i["iters"] for i in inf_e]
    eager.close()
    graph.close()


def test_autotuned_variants_keep_parity(tmp_path, monkeypatch):
    monkeypatch.setenv("LS_AUTOTUNE_CACHE", str(tmp_path / "autotune.txt"))
    m = models.random_medium((24, 20, 18), seed=9, rel=0.1, aniso_background=True)
    ctx = lsvie.context_from_model(m, omegas=[W], precision="mixed", max_rhs=2, autotune=True)
    v = ctx.kernel_variants
    sched = ctx.kernel_schedule
    print("variants", v, "schedule", sched, flush=True)
    assert set(v) == {"c128", "c64"} and all(len(x) == 5 for x in v.values())
    assert all(1 <= x["xy_chunk"] <= 2 for x in sched.values())
    P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, W)
    u = np.stack([models.random_field(m.shape, s) for s in range(2)])
    got = ctx.apply(torch.from_numpy(u)).cpu().numpy()
    got32 = ctx.apply(torch.from_numpy(u).to(torch.complex64)).cpu().numpy()
    for r in range(2):
        want = P.apply_fft(u[r])
        assert rel(got[r], want) < 1e-10
        assert rel(got32[r], want) < 1e-5
    ctx.close()


def test_solve_batch_over_uneven_grids():
    """Jobs over two contexts with different grids, frequency sets and max_rhs, interleaved in the job
    list (one frequency group larger than max_rhs): every job equals its own single solve; one equals the
    oracle's dense solve; the mixed-precision batch meets tol; bad jobs are refused before any work."""
    from oracle import solve
    ma = models.random_medium((14, 12, 10), seed=21, rel=0.1, aniso_background=True)
    mb = models.random_medium((20, 18, 16), seed=22, rel=0.1)
    wa = [2 * np.pi * 11.0, 2 * np.pi * 23.0]
    wb = [2 * np.pi * 17.0]
    A = lsvie.context_from_model(ma, omegas=wa, precision="mixed", max_rhs=2)
    B = lsvie.context_from_model(mb, omegas=wb, precision="mixed", max_rhs=3)
    dcpl = models.double_couple(30, 60, 90)
    jobs = [(0, 0, models.EXPLOSION, (7, 6, 5), 0.0), (1, 0, dcpl, (10, 9, 8), 0.002),
            (0, 1, dcpl, (3, 4, 2), 0.004), (0, 0, np.eye(6)[3], (0, 11, 9), 0.0),
            (1, 0, np.eye(6)[0], (19, 0, 15), 0.0), (0, 0, dcpl, (7, 6, 5), 0.001)]
    tol = 1e-11
    outs, infos = lsvie.solve_batch([A, B], jobs, tol=tol, maxit=2000, precision="c128")
    for (ci, iw, M, src, t0), u, info in zip(jobs, outs, infos):
        ctx = (A, B)[ci]
        want, _ = ctx.solve(ctx.rhs_moment(M, src, i_omega=iw, t0=t0), i_omega=iw, tol=tol, precision="c128")
        assert info["status"] == 0 and info["rel_res_true"] <= tol
        assert rel(u.cpu().numpy(), want.cpu().numpy()) < 1e-9, (ci, iw, src)
    P = op.Problem(ma.shape, ma.h, ma.C0, ma.rho0, ma.dc21, ma.drho, wa[1])
    dense = solve.solve_dense(P.dense_A(), P.rhs_moment(dcpl, (3, 4, 2), 0.004))
    assert rel(outs[2].cpu().numpy(), dense) < 1e-9
    outs_m, infos_m = lsvie.solve_batch([A, B], jobs, tol=1e-7, precision="mixed")
    for u, um, info in zip(outs, outs_m, infos_m):
        assert info["status"] == 0 and info["rel_res_true"] <= 1e-7
        assert rel(um.cpu().numpy(), u.cpu().numpy()) < 1e-5
    with pytest.raises(lsvie.LsError) as e:
        lsvie.solve_batch([A, B], [(1, 0, dcpl, (20, 0, 0), 0.0)])
    assert e.value.code == lsvie.LS_ERR_ARG
    with pytest.raises(lsvie.LsError) as e:
        lsvie.solve_batch([A, B], [(0, 2, dcpl, (1, 1, 1), 0.0)])
    assert e.value.code == lsvie.LS_ERR_ARG
    A.close()
    B.close()


def test_autotune_cache_is_written_and_used(tmp_path, monkeypatch):
    """The first tuned context writes its choice under its key; a context of the same configuration takes
    the cached choice without timing, here an edited line selecting the LDS Stockham kernels everywhere,
    and keeps parity with the oracle."""
    cache = tmp_path / "autotune.txt"
    monkeypatch.setenv("LS_AUTOTUNE_CACHE", str(cache))
    m = models.random_medium((16, 12, 10), seed=19, rel=0.1, aniso_background=True)
    ctx = lsvie.context_from_model(m, omegas=[W], precision="mixed", max_rhs=2, autotune=True)
    ctx.close()
    lines = cache.read_text().split("\n")
    key, *vals = lines[0].split()
    # ten kernel variants, then per precision the x/y chunk (1 .. max_rhs) and the strided tile choice
    assert len(vals) == 14 and set(vals[:10]) <= {"0", "1"} and key.startswith("v2:")
    assert all(1 <= int(x) <= 2 for x in vals[10:12]) and set(vals[12:]) <= {"0", "1"}
    cache.write_text(lines[0] + "\n" + key + " 1 1 1 1 1 1 1 1 1 1 1 1 0 0\n")
    ctx = lsvie.context_from_model(m, omegas=[W], precision="mixed", max_rhs=2, autotune=True)
    v = ctx.kernel_variants
    assert all(x == "stockham" for p in v.values() for x in p.values()), v
    assert ctx.kernel_schedule == {p: {"xy_chunk": 1, "wide_y_tiles": False} for p in ("c128", "c64")}
    P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, W)
    u = models.random_field(m.shape, 3)
    assert rel(ctx.apply(torch.from_numpy(u)).cpu().numpy(), P.apply_fft(u)) < 1e-10
    assert rel(ctx.apply(torch.from_numpy(u).to(torch.complex64)).cpu().numpy(), P.apply_fft(u)) < 1e-5
    ctx.close()
    assert len(cache.read_text().strip().split("\n")) == 2   # the cached key was not tuned again
    # on a grid whose y pass (length 64) can take 256-byte tiles, a register-kernel schedule with one-system
    # chunks and 128-byte tiles gives bitwise the same applies as the default schedule (two-system chunks, wide
    # tiles): the chunks and tiles regroup the same per-line transforms
    m2 = models.random_medium((16, 32, 10), seed=23, rel=0.1)
    t = lsvie.context_from_model(m2, omegas=[W], precision="mixed", max_rhs=2, autotune=True)
    t.close()
    key2 = cache.read_text().strip().split("\n")[-1].split()[0]
    cache.write_text(key2 + " 0 0 0 0 0 0 0 0 0 0 1 1 0 0\n")
    ctx = lsvie.context_from_model(m2, omegas=[W], precision="mixed", max_rhs=2, autotune=True)
    ref = lsvie.context_from_model(m2, omegas=[W], precision="mixed", max_rhs=2)
    assert ctx.kernel_schedule == {p: {"xy_chunk": 1, "wide_y_tiles": False} for p in ("c128", "c64")}
    assert ref.kernel_schedule == {p: {"xy_chunk": 2, "wide_y_tiles": True} for p in ("c128", "c64")}
    u2 = torch.from_numpy(np.stack([models.random_field(m2.shape, s) for s in (4, 5)]))
    for dt in (torch.complex128, torch.complex64):
        assert torch.equal(ctx.apply(u2.to(dt)), ref.apply(u2.to(dt)))
    ctx.close()
    ref.close()


def test_autotuned_schedule_at_128_cubed_keeps_parity(tmp_path, monkeypatch):
    """At the benchmark's 128^3 grid, where the x and y passes run in cache-sized chunks, the autotuner's choice
    of kernel variants, y tiles and chunk (six right-hand sides) keeps the full-field parity with the oracle's
    FFT apply in both precisions."""
    monkeypatch.setenv("LS_AUTOTUNE_CACHE", str(tmp_path / "autotune.txt"))
    m = models.config3()
    w = m.omegas[-1]
    ctx = lsvie.context_from_model(m, omegas=[w], precision="mixed", max_rhs=6, autotune=True)
    sched = ctx.kernel_schedule
    print("variants", ctx.kernel_variants, "schedule", sched, flush=True)
    assert all(1 <= x["xy_chunk"] <= 6 for x in sched.values())
    u = np.stack([models.random_field(m.shape, s) for s in (61, 62, 63)])
    ut = torch.from_numpy(u)
    got = ctx.apply(ut).cpu().numpy()
    got32 = ctx.apply(ut.to(torch.complex64)).cpu().numpy()
    ctx.close()
    P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, w)
    P.table()
    for r in range(3):
        want = P.apply_fft(u[r])
        assert rel(got[r], want) < 1e-10 and rel(got32[r], want) < 1e-5
