"""The seeded input generators: determinism and the values their recipes fix."""

import numpy as np

from paper_2301_12836_amd import models


def test_double_couple_30_60_90():
    M = models.double_couple(30, 60, 90)
    expect = [-0.2165063509, -0.6495190528, 0.8660254038, -0.4330127019, 0.25, 0.375]
    assert np.allclose(M, expect, atol=1e-9)
    assert abs(M[:3].sum()) < 1e-15


def test_thomsen_vti_values():
    C = models.vti_from_thomsen(**models.VTI_CFG2)
    assert np.isclose(C[2, 2], 2.16e10) and np.isclose(C[3, 3], 6.936e9)
    assert np.isclose(C[0, 0], 2.592e10) and np.isclose(C[5, 5], 8.04576e9)
    assert np.isclose(C[0, 2], 8.77091e9, rtol=1e-6) and np.isclose(C[0, 1], 9.82848e9)


def test_rotation_preserves_invariants():
    C = models.vti_from_thomsen(**models.VTI_CFG2)
    R = models.rot_z(45.0) @ models.rot_y(30.0)
    Ct = models.rotate_voigt(C, R)
    # Kelvin-form eigenvalues (shear rows scaled by sqrt 2) are rotation invariant
    S = np.diag([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])
    assert np.allclose(np.linalg.eigvalsh(S @ C @ S), np.linalg.eigvalsh(S @ Ct @ S), rtol=1e-12)
    assert np.allclose(models.rotate_voigt(Ct, R.T), C, rtol=0, atol=1e-4)


def test_generators_are_deterministic():
    a, b = models.config3(n=16), models.config3(n=16)
    assert np.array_equal(a.dc21, b.dc21) and np.array_equal(a.drho, b.drho)
    c, d = models.config2(n=12), models.config2(n=12)
    assert np.array_equal(c.dc21, d.dc21)
    assert np.array_equal(models.random_field((4, 5, 6), 3), models.random_field((4, 5, 6), 3))


def test_config1_inclusion():
    m = models.config1()
    assert m.shape == (16, 16, 16) and m.sources[0][1] == (4, 8, 8)
    assert int((m.drho > 0).sum()) == 280
    assert np.isclose(m.drho.max(), 120.0)


def test_random_fields_are_normalised():
    g = models.gaussian_random_fields(np.random.default_rng(0), 2, 32, 8.0, 40.0)
    assert np.allclose(g.mean(axis=(1, 2, 3)), 0, atol=1e-12)
    assert np.allclose(g.std(axis=(1, 2, 3)), 1, atol=1e-12)


def test_anisotropic_double_couple():
    """C : sym(nu x d) reduces to mu x potency x the Aki-Richards double couple for isotropic C (the fault
    normal and slip are orthonormal, so the trace term vanishes); in a VTI medium it is no longer
    trace-free for an inclined fault."""
    for sdr in ((30, 60, 90), (0, 90, 0), (120, 35, -45)):
        nu, d = models.fault_vectors(*sdr)
        assert np.isclose(nu @ nu, 1) and np.isclose(d @ d, 1) and abs(nu @ d) < 1e-14
        Ciso = models.iso_C(3000.0, 1700.0, 2400.0)
        mu = Ciso[3, 3]
        M = models.double_couple_aniso(Ciso, *sdr, potency=2.0)
        assert np.allclose(M, models.double_couple(*sdr, m0=2.0 * mu), rtol=1e-12, atol=1e-3)
    Cvti = models.vti_from_thomsen(**models.VTI_CFG2)
    M = models.double_couple_aniso(Cvti, 30, 60, 90)
    assert abs(M[0] + M[1] + M[2]) > 1e-3 * np.abs(M).max()


def test_paper_model2_layers_and_backgrounds():
    """Model 2: layer k takes the printed stiffness of the layer holding depth k h (boundaries at 108 and
    212 m); both backgrounds give the same total stiffness, and the mean background is the thickness mean."""
    mid = models.paper_model2(n=128, h=2.5)
    mean = models.paper_model2(n=128, h=2.5, background="mean")
    layers = [models.vti_C(*(1e9 * np.array(p))) for p in models.PAPER_MODEL2_LAYERS]
    for k, L in ((0, 0), (43, 0), (44, 1), (84, 1), (85, 2), (127, 2)):   # 43*2.5 = 107.5, 85*2.5 = 212.5
        want = models.pack21(layers[L])
        assert np.allclose(mid.dc21[:, k, 5, 7] + models.pack21(mid.C0), want, rtol=0, atol=1.0)
        assert np.allclose(mean.dc21[:, k, 3, 9] + models.pack21(mean.C0), want, rtol=0, atol=1.0)
    assert np.array_equal(mid.C0, layers[1]) and not mid.dc21[:, 60].any()
    assert np.allclose(mean.C0, (108 * layers[0] + 104 * layers[1] + 108 * layers[2]) / 320, rtol=1e-14)
    assert mean.rho0 == 2500.0 and not mean.drho.any() and mid.sources[0][1] == (64, 64, 64)
