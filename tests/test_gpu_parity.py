"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle, element by element.

Bars: the FP64 (c128) operator within relative L2 1e-10 of the oracle; the FP32 (c64) operator and
the mixed-precision solve within 1e-5; integer-free, so no bit-exact cases except the batched-vs-
single comparison, which must be bitwise identical.
"""

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


def ctx_and_problem(m, omegas=None, precision="c128", max_rhs=1, mode="exact"):
    omegas = m.omegas if omegas is None else omegas
    ctx = lsvie.context_from_model(m, precision=precision, max_rhs=max_rhs, omegas=omegas, green_mode=mode)
    P = [op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, w, mode=mode) for w in omegas]
    return ctx, P


def to_np(t):
    return t.detach().cpu().numpy()


SHAPES = [(16, 16, 16), (12, 9, 7), (5, 6, 4), (2, 3, 2), (17, 8, 11)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("aniso", [False, True])
def test_apply_c128_matches_oracle(shape, aniso):
    m = models.random_medium(shape, seed=sum(shape), rel=0.1, aniso_background=aniso)
    ctx, (P,) = ctx_and_problem(m, omegas=[W15])
    u = models.random_field(shape, seed=3)
    got = to_np(ctx.apply(torch.from_numpy(u)))
    want = P.apply_fft(u)
    print("shape", shape, "aniso", aniso, "rel", rel(got, want), flush=True)
    assert rel(got, want) < 1e-10
    ctx.close()


@pytest.mark.parametrize("mode", ["exact", "paper_sum"])
def test_apply_config1_both_green_modes(mode):
    m = models.config1()
    ctx, (P,) = ctx_and_problem(m, mode=mode)
    u = models.random_field(m.shape, seed=5)
    got = to_np(ctx.apply(torch.from_numpy(u)))
    assert rel(got, P.apply_fft(u)) < 1e-10
    # direct per-cell sums at a few cells (independent of any FFT)
    cells = np.array([[0, 0, 0], [15, 15, 15], [4, 8, 8], [7, 3, 12]])
    direct = P.apply_bruteforce(u, cells)
    assert rel(got[:, cells[:, 2], cells[:, 1], cells[:, 0]].T, direct) < 1e-10
    ctx.close()


def test_apply_c64_matches_oracle():
    m = models.random_medium((16, 12, 10), seed=2, rel=0.1, aniso_background=True)
    ctx, (P,) = ctx_and_problem(m, omegas=[W15], precision="mixed")
    u = models.random_field(m.shape, seed=7)
    got = to_np(ctx.apply(torch.from_numpy(u).to(torch.complex64)))
    want = P.apply_fft(u)
    print("c64 rel", rel(got, want), flush=True)
    assert rel(got, want) < 1e-5
    ctx.close()


def test_batched_apply_is_bitwise_equal_to_single():
    m = models.random_medium((12, 10, 9), seed=4, rel=0.1)
    ctx, _ = ctx_and_problem(m, omegas=[W15, 2 * W15], max_rhs=4)
    u = torch.from_numpy(np.stack([models.random_field(m.shape, seed=s) for s in range(4)]))
    for iw in range(2):
        batch = to_np(ctx.apply(u, i_omega=iw))
        for r in range(4):
            single = to_np(ctx.apply(u[r], i_omega=iw))
            assert np.array_equal(batch[r], single)
    ctx.close()


@pytest.mark.parametrize("src", [(4, 8, 8), (0, 3, 15), (15, 0, 7), (1, 14, 1)])
def test_rhs_moment_matches_oracle(src):
    m = models.config1()
    ctx, (P,) = ctx_and_problem(m)
    M = np.array([0.3, -1.1, 0.7, 0.25, -0.4, 0.9])
    got = to_np(ctx.rhs_moment(M, src, t0=0.013))
    want = P.rhs_moment(M, src, t0=0.013)
    assert rel(got, want) < 1e-12
    ctx.close()


def test_rhs_force_matches_oracle():
    m = models.random_medium((9, 7, 8), seed=1)
    ctx, (P,) = ctx_and_problem(m, omegas=[W15])
    got = to_np(ctx.rhs_force([0.2, -1.0, 0.5], (3, 2, 6)))
    assert rel(got, P.rhs_force([0.2, -1.0, 0.5], (3, 2, 6))) < 1e-12
    ctx.close()


def test_zero_contrast_apply_is_identity_and_solve_returns_rhs():
    shape = (10, 10, 10)
    C0 = models.iso_C(3000.0, 1730.0, 2400.0)
    m = models.Model(shape, 10.0, C0, 2400.0, np.zeros((21, 10, 10, 10)), np.zeros((10, 10, 10)), [15.0])
    ctx, _ = ctx_and_problem(m)
    u = models.random_field(shape, 9)
    assert np.array_equal(to_np(ctx.apply(torch.from_numpy(u))), u), "A must be the identity"
    b = ctx.rhs_moment(models.EXPLOSION, (5, 5, 5))
    x, infos = ctx.solve(b, tol=1e-10)
    # A = I: the first half step gives s = r - A r = 0, so x = b after one iteration
    assert bool(torch.equal(x, b)), "zero-contrast solve must return the incident field"
    assert infos[0]["iters"] == 1 and infos[0]["rel_res_true"] == 0.0
    ctx.close()


def test_strain_matches_oracle():
    m = models.random_medium((7, 9, 6), seed=3)
    ctx, _ = ctx_and_problem(m, omegas=[W15])
    u = models.random_field(m.shape, 2)
    got = to_np(ctx.strain(torch.from_numpy(u)))
    assert rel(got, op.strain_apply(u, m.h)) < 1e-13
    ctx.close()


def test_solve_c128_matches_lu():
    m = models.config1(n=10)
    ctx, (P,) = ctx_and_problem(m)
    b = ctx.rhs_moment(models.EXPLOSION, (3, 5, 5))
    x, infos = ctx.solve(b, tol=1e-12, maxit=500)
    want = solve.solve_dense(P.dense_A(), P.rhs_moment(models.EXPLOSION, (3, 5, 5)))
    print("solve rel", rel(to_np(x), want), infos, flush=True)
    assert rel(to_np(x), want) < 1e-10
    assert infos[0]["rel_res_true"] < 1e-11
    ctx.close()


def test_solve_config1_c128_and_mixed():
    """Config 1 (16^3, tol 1e-8): GPU solves against the oracle's BiCGSTAB to 1e-13 on its FFT operator."""
    m = models.config1()
    ctx, (P,) = ctx_and_problem(m, precision="mixed")
    M, src = m.sources[0]
    want, hist, _ = solve.bicgstab(P.apply_fft, P.rhs_moment(M, src), 1e-13, 1000)
    b = ctx.rhs_moment(M, src)
    x, infos = ctx.solve(b, tol=1e-8, precision="c128")
    e128 = rel(to_np(x), want)
    x32, infos32 = ctx.solve(b, tol=1e-8, precision="mixed")
    e_mixed = rel(to_np(x32), want)
    print("config1 c128", e128, infos, "mixed", e_mixed, infos32, flush=True)
    assert infos[0]["rel_res_true"] <= 1e-8 and e128 < 1e-6
    assert infos32[0]["rel_res_true"] <= 1e-8 and e_mixed < 1e-6
    # the oracle certifies the GPU solution's residual on its own operator
    assert solve.relative_residual(P.apply_fft, to_np(x), P.rhs_moment(M, src)) < 2e-8
    ctx.close()


def test_solve_batch_of_moment_tensors():
    m = models.random_medium((12, 12, 12), seed=8, rel=0.08, aniso_background=True)
    ctx, (P,) = ctx_and_problem(m, omegas=[W15], precision="mixed", max_rhs=6)
    src = (6, 5, 7)
    bs = torch.stack([ctx.rhs_moment(np.eye(6)[J], src) for J in range(6)])
    x, infos = ctx.solve(bs, tol=1e-9, precision="c128")
    xm, infos_m = ctx.solve(bs, tol=1e-6, precision="mixed")
    for J in range(6):
        bJ = P.rhs_moment(np.eye(6)[J], src)
        assert solve.relative_residual(P.apply_fft, to_np(x[J]), bJ) < 1e-8
        assert solve.relative_residual(P.apply_fft, to_np(xm[J]), bJ) < 1.5e-6
        assert rel(to_np(xm[J]), to_np(x[J])) < 1e-5
    # linearity in M: u(M) = sum_J M_J u(e_J)
    M = models.double_couple(30, 60, 90)
    xM, _ = ctx.solve(ctx.rhs_moment(M, src), tol=1e-9, precision="c128")
    comb = np.tensordot(M, to_np(x), axes=(0, 0))
    assert rel(to_np(xM), comb) < 1e-7
    ctx.close()


def test_reciprocity_on_gpu():
    m = models.random_medium((8, 9, 7), seed=5, rel=0.1, aniso_background=True)
    ctx, _ = ctx_and_problem(m, omegas=[W15])
    r, s = (1, 2, 4), (6, 5, 2)
    sol = {}
    for cell in (r, s):
        for c in range(3):
            x, _ = ctx.solve(ctx.rhs_force(np.eye(3)[c], cell), tol=1e-12, maxit=800)
            sol[cell, c] = to_np(x)
    for i in range(3):
        for j in range(3):
            a = sol[s, j][i, r[2], r[1], r[0]]
            b = sol[r, i][j, s[2], s[1], s[0]]
            assert abs(a - b) < 1e-9 * max(abs(a), abs(b))
    ctx.close()


def test_error_paths_on_gpu():
    m = models.random_medium((6, 6, 6), seed=1)
    ctx, _ = ctx_and_problem(m, omegas=[W15])
    b = ctx.rhs_moment(models.EXPLOSION, (3, 3, 3))
    with pytest.raises(lsvie.LsError) as e:
        ctx.solve(b, tol=1e-12, maxit=1)
    assert e.value.code == lsvie.LS_ERR_NOT_CONVERGED
    with pytest.raises(lsvie.LsError) as e:
        ctx.rhs_moment(models.EXPLOSION, (6, 0, 0))
    assert e.value.code == lsvie.LS_ERR_ARG
    with pytest.raises(lsvie.LsError) as e:
        ctx.apply(torch.zeros((3, 6, 6, 6), dtype=torch.complex64))
    assert e.value.code == lsvie.LS_ERR_STATE
    with pytest.raises(lsvie.LsError):
        ctx.apply(torch.from_numpy(models.random_field(m.shape, 1)), i_omega=3)
    # outputs of the wrong element type or shape are refused before anything is launched
    u128 = torch.from_numpy(models.random_field(m.shape, 1)).to(ctx.device)
    for call in (ctx.apply, ctx.apply_T, ctx.convolve):
        with pytest.raises(ValueError):
            call(u128, out=torch.empty(u128.shape, dtype=torch.complex64, device=ctx.device))
        with pytest.raises(ValueError):
            call(u128, out=torch.empty((2,) + u128.shape, dtype=torch.complex128, device=ctx.device))
    with pytest.raises(ValueError):
        ctx.solve(b, out=torch.empty(b.shape, dtype=torch.complex64, device=ctx.device))
    with pytest.raises(ValueError):
        ctx.rhs_moment(models.EXPLOSION, (3, 3, 3), out=torch.empty((1, 1), dtype=torch.complex128,
                                                                    device=ctx.device))
    # an empty batch and one beyond max_rhs (1 here) are refused by the library: n_rhs outside [1, max_rhs]
    for nr in (0, 2):
        for call in (ctx.apply, ctx.solve):
            with pytest.raises(lsvie.LsError) as e:
                call(torch.zeros((nr,) + tuple(b.shape), dtype=torch.complex128, device=ctx.device))
            assert e.value.code == lsvie.LS_ERR_ARG
    # zero right-hand side: immediate u = 0
    x, infos = ctx.solve(torch.zeros_like(b), tol=1e-8)
    assert float(torch.abs(x).max()) == 0.0 and infos[0]["iters"] == 0
    ctx.close()


def test_apply_config2_full_field_c128_and_c64():
    """64^3 layered VTI (FFT length 128): full-field parity of both operator precisions."""
    m = models.config2()
    ctx, (P,) = ctx_and_problem(m, precision="mixed")
    u = models.random_field(m.shape, seed=11)
    want = P.apply_fft(u)
    got = to_np(ctx.apply(torch.from_numpy(u)))
    got32 = to_np(ctx.apply(torch.from_numpy(u).to(torch.complex64)))
    print("config2 c128", rel(got, want), "c64", rel(got32, want), flush=True)
    assert rel(got, want) < 1e-10
    assert rel(got32, want) < 1e-5
    ctx.close()


def test_apply_config3_sampled_cells_batched():
    """128^3 TTI random medium, 6 right-hand sides in one launch (the benchmark's configuration):
    sampled output cells against the oracle's direct per-cell sums."""
    m = models.config3()
    omega = m.omegas[-1]
    ctx = lsvie.context_from_model(m, precision="mixed", max_rhs=6, omegas=[omega])
    P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, omega)
    rng = np.random.default_rng(5)
    cells = np.concatenate([rng.integers(0, 128, size=(4, 3)), [[0, 0, 0], [127, 127, 127], [64, 64, 64]]])
    u = np.stack([models.random_field(m.shape, seed=s) for s in range(6)])
    got = to_np(ctx.apply(torch.from_numpy(u)))
    got32 = to_np(ctx.apply(torch.from_numpy(u).to(torch.complex64)))
    for r in (0, 5):
        want = P.apply_bruteforce(u[r], cells)
        g = got[r][:, cells[:, 2], cells[:, 1], cells[:, 0]].T
        g32 = got32[r][:, cells[:, 2], cells[:, 1], cells[:, 0]].T
        print("config3 rhs", r, "c128", rel(g, want), "c64", rel(g32, want), flush=True)
        assert rel(g, want) < 1e-10
        assert rel(g32, want) < 1e-5
    ctx.close()


@pytest.mark.parametrize("shape", [(20, 24, 40), (17, 40, 9), (48, 33, 10)])
def test_radix3_lengths_match_oracle(shape):
    """Grids whose padded FFT lengths carry a factor 3 (48, 96) on some axes and are powers of two on
    others: c128 and c64 applies against the oracle (which pads to 2N independently)."""
    m = models.random_medium(shape, seed=sum(shape) + 3, rel=0.1, aniso_background=True)
    w = 2 * np.pi * 18.0
    ctx, (P,) = ctx_and_problem(m, omegas=[w], precision="mixed")
    u = models.random_field(shape, 4)
    want = P.apply_fft(u)
    got = to_np(ctx.apply(torch.from_numpy(u)))
    got32 = to_np(ctx.apply(torch.from_numpy(u).to(torch.complex64)))
    print(shape, "c128", rel(got, want), "c64", rel(got32, want), flush=True)
    assert rel(got, want) < 1e-10
    assert rel(got32, want) < 1e-5
    ctx.close()


def test_absorbing_taper_apply_and_gradient_weight():
    """The absorbing layer (Eq 23-25) against the oracle's tapered problem, and the gradient's chain rule
    through the weight: with the same fields, tapered gradients are the oracle's weights times untapered."""
    m = models.random_medium((14, 12, 10), seed=31, rel=0.1, aniso_background=True)
    d = 3
    ctx = lsvie.context_from_model(m, omegas=[W15], precision="mixed", taper=d)
    P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, W15, taper=d)
    u = models.random_field(m.shape, 8)
    want = P.apply_fft(u)
    assert rel(to_np(ctx.apply(torch.from_numpy(u))), want) < 1e-10
    assert rel(to_np(ctx.apply(torch.from_numpy(u).to(torch.complex64))), want) < 1e-5
    ctx0 = lsvie.context_from_model(m, omegas=[W15])
    mu = torch.from_numpy(models.random_field(m.shape, 9))
    g, gr = ctx.grad_contrast(torch.from_numpy(u), mu)
    g0, gr0 = ctx0.grad_contrast(torch.from_numpy(u), mu)
    w = op.taper_weights(m.shape, d)
    assert np.allclose(to_np(g), w[None] * to_np(g0), rtol=1e-13, atol=0)
    assert np.allclose(to_np(gr), w * to_np(gr0), rtol=1e-13, atol=0)
    ctx.close()
    ctx0.close()
    with pytest.raises(lsvie.LsError) as e:
        lsvie.context_from_model(m, omegas=[W15], taper=6)
    assert e.value.code == lsvie.LS_ERR_ARG


def test_residual_history_matches_textbook_bicgstab():
    """The recorded residual after each iteration equals the oracle's textbook BiCGSTAB on the same system
    (same iterates in exact arithmetic: x0 = 0, shadow residual r0) while rounding is small, and the
    mixed-precision record (inner residuals scaled to the original system) ends below tol."""
    from oracle import solve
    m = models.random_medium((8, 7, 6), seed=12, rel=0.1, aniso_background=True)
    ctx, (P,) = ctx_and_problem(m, omegas=[W15], precision="mixed")
    b = ctx.rhs_moment(models.EXPLOSION, (4, 3, 3))
    x, infos = ctx.solve(b, tol=1e-10, precision="c128")
    h = ctx.residual_history(0)
    _, hist, _ = solve.bicgstab(P.apply_fft, to_np(b), 1e-10)
    print("iterations", len(h), len(hist) - 1, "first", h[:4], hist[1:5], flush=True)
    assert len(h) == infos[0]["iters"] and abs(len(h) - (len(hist) - 1)) <= 1
    for i in range(min(5, len(h))):
        assert abs(h[i] - hist[i + 1]) <= 1e-8 * hist[i + 1]
    xm, im = ctx.solve(b, tol=1e-6, precision="mixed")
    hm = ctx.residual_history(0)
    assert len(hm) == im[0]["iters"] and hm[-1] < 1e-6 and hm[0] < 1.0
    with pytest.raises(lsvie.LsError):
        ctx.residual_history(1)
    ctx.close()


def test_nonfinite_contrast_is_reported():
    m = models.random_medium((6, 6, 6), seed=2)
    dc = m.dc21.copy()
    dc[0, 3, 3, 3] = np.nan
    ctx = lsvie.Context(m.shape, m.h, m.C0, m.rho0, dc, m.drho, [W15], precision="mixed")
    b = ctx.rhs_moment(models.EXPLOSION, (2, 2, 2))
    for prec in ("c128", "mixed"):
        _, infos = ctx.solve(b, tol=1e-8, precision=prec, raise_on_error=False)
        assert infos[0]["status"] == lsvie.LS_ERR_NONFINITE, (prec, infos)
    with pytest.raises(lsvie.LsError) as e:
        ctx.solve(b, tol=1e-8, precision="c128")
    assert e.value.code == lsvie.LS_ERR_NONFINITE
    ctx.close()


@pytest.mark.parametrize("shape", [(12, 9, 16), (8, 8, 64)])
def test_blocked_work_layout_matches_oracle(shape, monkeypatch):
    """The work buffer with z planes interleaved in blocks of 8 (the layout the library takes where the z
    line is 512 long), forced at small sizes: 16 planes run the LDS z kernel, 64 the register kernel.
    Apply (c128 and c64), transposed apply and Green's convolution against the oracle, and the blocked
    c128 apply against the plain one."""
    from oracle import adjoint as oadj
    m = models.random_medium(shape, seed=sum(shape), rel=0.1, aniso_background=True)
    P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, W15)
    u = models.random_field(shape, seed=3)
    ut = torch.from_numpy(u)
    monkeypatch.setenv("LS_ZBLOCK", "0")
    plain = lsvie.context_from_model(m, omegas=[W15], precision="mixed", max_rhs=2)
    want_plain = to_np(plain.apply(ut))
    plain.close()
    monkeypatch.setenv("LS_ZBLOCK", "8")
    ctx = lsvie.context_from_model(m, omegas=[W15], precision="mixed", max_rhs=2)
    got = to_np(ctx.apply(ut))
    got32 = to_np(ctx.apply(ut.to(torch.complex64)))
    want = P.apply_fft(u)
    print(shape, "c128", rel(got, want), "c64", rel(got32, want), "vs plain", rel(got, want_plain), flush=True)
    assert rel(got, want) < 1e-10 and rel(got32, want) < 1e-5
    assert rel(got, want_plain) < 1e-13
    assert rel(to_np(ctx.apply_T(ut)), oadj.apply_T(P, u)) < 1e-10
    assert rel(to_np(ctx.convolve(ut)), op.convolve_fft(u, P.table())) < 1e-10
    # two right-hand sides in one launch: the blocked rows of both are kept apart
    u2 = torch.stack([ut, torch.from_numpy(models.random_field(shape, seed=4))])
    got2 = to_np(ctx.apply(u2))
    assert rel(got2[0], want) < 1e-10 and rel(got2[1], P.apply_fft(to_np(u2[1]))) < 1e-10
    ctx.close()


@pytest.mark.parametrize("zblock", ["0", "8"])
def test_z_length_512_matches_oracle(zblock, monkeypatch):
    """A z line of 512 padded points (8 x 8 x 256 cells): the paired register z pass (32 threads of 16
    values per line) in both precisions, with the blocked and the plain work-buffer layout."""
    monkeypatch.setenv("LS_ZBLOCK", zblock)
    shape = (8, 8, 256)
    m = models.random_medium(shape, seed=5, rel=0.1)
    P = op.Problem(m.shape, m.h, m.C0, m.rho0, m.dc21, m.drho, W15)
    ctx = lsvie.context_from_model(m, omegas=[W15], precision="mixed", max_rhs=2)
    u = models.random_field(shape, seed=6)
    ut = torch.from_numpy(u)
    want = P.apply_fft(u)
    got = to_np(ctx.apply(ut))
    got32 = to_np(ctx.apply(ut.to(torch.complex64)))
    print("zblock", zblock, "c128", rel(got, want), "c64", rel(got32, want), ctx.kernel_variants, flush=True)
    assert rel(got, want) < 1e-10 and rel(got32, want) < 1e-5
    u2 = torch.stack([ut, torch.from_numpy(models.random_field(shape, seed=7))])
    got2 = to_np(ctx.apply(u2.to(torch.complex64)))
    assert rel(got2[1], P.apply_fft(to_np(u2[1]))) < 1e-5
    ctx.close()
