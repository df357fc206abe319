"""Seeded synthetic inputs shaped like the paper's models (input generation only).

This module draws media, sources and frequencies; it holds none of the LS
method's arithmetic (no Green's tensor, strain stencil, contrast product or
background folding), so both the HIP path and the CPU oracle take its arrays
as plain inputs.  All randomness comes from ``numpy.random.default_rng(seed)``.

Recipes (sizes, value ranges and structure mirror the paper's experiments):

* ``config1`` - 16^3, h = 10 m, isotropic background vp 3000, vs 1730, rho
  2400; sphere of radius 40 m at the grid centre with +10 % on the isotropic
  stiffness and +5 % density; 15 Hz; explosion M = diag(1,1,1) at cell (4,8,8).
* ``config2`` - 64^3, h = 10 m, VTI background from Thomsen parameters
  (vp0 3000, vs0 1700, eps 0.1, delta 0.05, gamma 0.08, rho 2400), three
  horizontal layers with uniform +-15 % on C11, C33, C44, C66, C13 (seed 1),
  20 Hz, double couple 30/60/90 at the centre (the layered VTI structure of the
  paper's Model 2).
* ``config3`` - 128^3, h = 8 m: config 2's VTI tilted 30 deg about y and
  rotated 45 deg about z (TTI), times (1 + 0.08 g_IJ(x)) on all 21 stiffnesses
  and rho = 2400 (1 + 0.04 g_rho(x)), g Gaussian random fields with covariance
  exp(-r^2/L^2), L = 40 m (seed 2), over an isotropic background (3000, 1700,
  2400); 6 elementary moment tensors x 8 frequencies 5-40 Hz at the centre.
  It stands in for the paper's Hess/SEG model, which is not available here.
* ``config4`` - 96^3 ellipsoid anomaly in config 2's VTI background.
* ``paper_model2`` - the paper's own Model 2 (Table 2 stiffnesses, 320 m cube, h = 2.5 m, three layers
  108 / 104 / 108 m thick, density 2500), for running the paper's workloads as printed.

Every function also takes ``n`` so the same recipe can be drawn at small sizes
for parity tests.
"""

from dataclasses import dataclass, field

import numpy as np

UPPER21 = tuple((I, J) for I in range(6) for J in range(I, 6))
VOIGT_PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


@dataclass
class Model:
    shape: tuple            # (N1, N2, N3) = (x, y, z)
    h: float
    C0: np.ndarray          # 6x6 background stiffness (Pa)
    rho0: float
    dc21: np.ndarray        # [21, N3, N2, N1] contrast relative to C0 (Pa)
    drho: np.ndarray        # [N3, N2, N1] density contrast (kg/m^3)
    freqs: list             # Hz
    sources: list = field(default_factory=list)   # [(M Voigt 11,22,33,23,13,12, (i, j, k))]
    tol: float = 1e-6
    name: str = ""

    @property
    def omegas(self):
        return [2.0 * np.pi * f for f in self.freqs]


def iso_C(vp, vs, rho):
    c11, c44 = rho * vp * vp, rho * vs * vs
    C = np.zeros((6, 6))
    C[:3, :3] = c11 - 2.0 * c44
    for I in range(3):
        C[I, I] = c11
        C[I + 3, I + 3] = c44
    return C


def vti_from_thomsen(vp0, vs0, eps, delta, gamma, rho):
    """Thomsen (1986) parameters -> VTI Voigt stiffness (symmetry axis z)."""
    c33 = rho * vp0 * vp0
    c44 = rho * vs0 * vs0
    c11 = c33 * (1.0 + 2.0 * eps)
    c66 = c44 * (1.0 + 2.0 * gamma)
    c13 = np.sqrt(2.0 * delta * c33 * (c33 - c44) + (c33 - c44) ** 2) - c44
    return vti_C(c11, c33, c44, c66, c13)


def vti_C(c11, c33, c44, c66, c13):
    C = np.zeros((6, 6))
    C[0, 0] = C[1, 1] = c11
    C[2, 2] = c33
    C[3, 3] = C[4, 4] = c44
    C[5, 5] = c66
    C[0, 1] = C[1, 0] = c11 - 2.0 * c66
    C[0, 2] = C[2, 0] = C[1, 2] = C[2, 1] = c13
    return C


def pack21(C66):
    C66 = np.asarray(C66)
    return np.stack([C66[I, J] for (I, J) in UPPER21])


def rotate_voigt(C, R):
    """Rotate a Voigt stiffness by the 3x3 rotation R: c'_ijkl = R_ip R_jq R_kr R_ls c_pqrs."""
    c = np.zeros((3, 3, 3, 3))
    for I, (i, j) in enumerate(VOIGT_PAIRS):
        for J, (k, l) in enumerate(VOIGT_PAIRS):
            for (a, b) in {(i, j), (j, i)}:
                for (p, q) in {(k, l), (l, k)}:
                    c[a, b, p, q] = C[I, J]
    cr = np.einsum('ip,jq,kr,ls,pqrs->ijkl', R, R, R, R, c)
    out = np.zeros((6, 6))
    for I, (i, j) in enumerate(VOIGT_PAIRS):
        for J, (k, l) in enumerate(VOIGT_PAIRS):
            out[I, J] = cr[i, j, k, l]
    return out


def rot_y(deg):
    t = np.deg2rad(deg)
    return np.array([[np.cos(t), 0, np.sin(t)], [0, 1, 0], [-np.sin(t), 0, np.cos(t)]])


def rot_z(deg):
    t = np.deg2rad(deg)
    return np.array([[np.cos(t), -np.sin(t), 0], [np.sin(t), np.cos(t), 0], [0, 0, 1]])


def double_couple(strike, dip, rake, m0=1.0):
    """Aki-Richards double couple (x north, y east, z down) -> Voigt (11,22,33,23,13,12)."""
    f, d, l = np.deg2rad([strike, dip, rake])
    m11 = -(np.sin(d) * np.cos(l) * np.sin(2 * f) + np.sin(2 * d) * np.sin(l) * np.sin(f) ** 2)
    m22 = np.sin(d) * np.cos(l) * np.sin(2 * f) - np.sin(2 * d) * np.sin(l) * np.cos(f) ** 2
    m33 = np.sin(2 * d) * np.sin(l)
    m12 = np.sin(d) * np.cos(l) * np.cos(2 * f) + 0.5 * np.sin(2 * d) * np.sin(l) * np.sin(2 * f)
    m13 = -(np.cos(d) * np.cos(l) * np.cos(f) + np.cos(2 * d) * np.sin(l) * np.sin(f))
    m23 = -(np.cos(d) * np.cos(l) * np.sin(f) - np.cos(2 * d) * np.sin(l) * np.cos(f))
    return m0 * np.array([m11, m22, m33, m23, m13, m12])


def fault_vectors(strike, dip, rake):
    """Unit fault normal nu and slip direction d of Aki and Richards (x north, y east, z down)."""
    f, dl, l = np.deg2rad([strike, dip, rake])
    nu = np.array([-np.sin(dl) * np.sin(f), np.sin(dl) * np.cos(f), -np.cos(dl)])
    d = np.array([np.cos(l) * np.cos(f) + np.cos(dl) * np.sin(l) * np.sin(f),
                  np.cos(l) * np.sin(f) - np.cos(dl) * np.sin(l) * np.cos(f),
                  -np.sin(l) * np.sin(dl)])
    return nu, d


def double_couple_aniso(C, strike, dip, rake, potency=1.0):
    """Moment tensor of a shear dislocation (slip x area = potency) in a medium of stiffness C (6x6 Voigt):
    M = potency C : sym(nu (x) d), the double-couple source of an anisotropic medium (the paper's VTI
    example takes its source this way).  For isotropic C it is mu potency times the Aki-Richards double
    couple; in anisotropic media it has non-double-couple parts.  Voigt (11,22,33,23,13,12)."""
    nu, d = fault_vectors(strike, dip, rake)
    e = np.array([nu[0] * d[0], nu[1] * d[1], nu[2] * d[2], nu[1] * d[2] + nu[2] * d[1],
                  nu[0] * d[2] + nu[2] * d[0], nu[0] * d[1] + nu[1] * d[0]])   # engineering Voigt strain
    return potency * (np.asarray(C, dtype=np.float64) @ e)


EXPLOSION = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])


def gaussian_random_fields(rng, count, n, h, corr_len):
    """count fields on an n^3 grid, covariance exp(-r^2/L^2), zero mean and unit std each."""
    k = 2.0 * np.pi * np.fft.fftfreq(n, d=h)
    kz, ky, kx = np.meshgrid(k, k, k, indexing='ij')
    amp = np.exp(-(kx**2 + ky**2 + kz**2) * corr_len**2 / 8.0)   # sqrt of the spectrum exp(-k^2 L^2/4)
    out = np.empty((count, n, n, n))
    for c in range(count):
        w = rng.standard_normal((n, n, n))
        g = np.fft.ifftn(np.fft.fftn(w) * amp).real
        g -= g.mean()
        out[c] = g / g.std()
    return out


def _centre(n):
    return 0.5 * (n - 1)


def config1(n=16):
    h = 10.0
    rho0 = 2400.0
    C0 = iso_C(3000.0, 1730.0, rho0)
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing='ij')
    c = _centre(n)
    inside = ((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2) * h * h <= 40.0 ** 2
    dc = np.zeros((21, n, n, n))
    d21 = pack21(0.1 * C0)
    dc[:, inside] = d21[:, None]
    drho = np.where(inside, 0.05 * rho0, 0.0)
    src = (4 * n // 16, 8 * n // 16, 8 * n // 16)
    return Model((n, n, n), h, C0, rho0, dc, drho, [15.0], [(EXPLOSION.copy(), src)], 1e-8, "config1")


VTI_CFG2 = dict(vp0=3000.0, vs0=1700.0, eps=0.1, delta=0.05, gamma=0.08, rho=2400.0)


def config2(n=64, seed=1):
    h = 10.0
    rho0 = 2400.0
    C0 = vti_from_thomsen(**VTI_CFG2)
    rng = np.random.default_rng(seed)
    base = np.array([C0[0, 0], C0[2, 2], C0[3, 3], C0[5, 5], C0[0, 2]])
    bounds = [0, n // 3, 2 * n // 3, n]
    dc = np.zeros((21, n, n, n))
    for layer in range(3):
        p = base * (1.0 + rng.uniform(-0.15, 0.15, size=5))
        dC = vti_C(*p) - C0
        dc[:, bounds[layer]:bounds[layer + 1]] = pack21(dC)[:, None, None, None]
    drho = np.zeros((n, n, n))
    m = n // 2
    return Model((n, n, n), h, C0, rho0, dc, drho, [20.0], [(double_couple(30, 60, 90), (m, m, m))],
                 1e-6, "config2")


def tti_cfg3():
    C = vti_from_thomsen(**VTI_CFG2)
    return rotate_voigt(C, rot_z(45.0) @ rot_y(30.0))


def config3(n=128, seed=2, h=8.0, freqs=(5, 10, 15, 20, 25, 30, 35, 40)):
    rho0 = 2400.0
    C0 = iso_C(3000.0, 1700.0, rho0)
    Ct = tti_cfg3()
    rng = np.random.default_rng(seed)
    g = gaussian_random_fields(rng, 22, n, h, 40.0)
    ct21 = pack21(Ct)
    dc = ct21[:, None, None, None] * (1.0 + 0.08 * g[:21]) - pack21(C0)[:, None, None, None]
    drho = rho0 * 0.04 * g[21]
    m = n // 2
    sources = [(np.eye(6)[J], (m, m, m)) for J in range(6)]
    return Model((n, n, n), h, C0, rho0, dc, drho, list(map(float, freqs)), sources, 1e-6, "config3")


def config4(n=96):
    h = 10.0
    rho0 = 2400.0
    C0 = vti_from_thomsen(**VTI_CFG2)
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing='ij')
    c = _centre(n)
    inside = (((x - c) * h / 120.0) ** 2 + ((y - c) * h / 80.0) ** 2 + ((z - c) * h / 60.0) ** 2) <= 1.0
    dc = np.zeros((21, n, n, n))
    dC = np.zeros((6, 6))
    dC[2, 2] = 0.12 * C0[2, 2]
    dc[:, inside] = pack21(dC)[:, None]
    drho = np.where(inside, -0.08 * rho0, 0.0)
    zs = 60 * n // 96
    srcs = [(EXPLOSION.copy(), (32 * n // 96, 48 * n // 96, zs)),
            (double_couple(30, 60, 90), (48 * n // 96, 48 * n // 96, zs)),
            (double_couple(0, 90, 0), (64 * n // 96, 48 * n // 96, zs))]
    return Model((n, n, n), h, C0, rho0, dc, drho, [8.0, 16.0, 24.0, 32.0], srcs, 1e-6, "config4")


def config4_receivers(n=96):
    """64 receivers on a surface line: z = 0, y = n/2, x = n/6 ... n/6 + 63 (clipped to the grid)."""
    x0 = 16 * n // 96
    xs = [min(x0 + i, n - 1) for i in range(64)] if n >= 80 else list(range(0, n, max(1, n // 8)))
    return np.array([[x, 48 * n // 96, 0] for x in xs])


def config4_observed(n=96, seed=3):
    """The 'true' model whose data the misfit compares against: config 4's ellipsoid with its C33 and
    rho anomalies each scaled by (1 + 0.25 xi), xi uniform in [-1, 1] (seed 3), plus a 2 % random
    perturbation of C33 and rho inside the ellipsoid."""
    m = config4(n)
    rng = np.random.default_rng(seed)
    a, b = 1.0 + 0.25 * rng.uniform(-1, 1, size=2)
    inside = m.drho != 0.0
    q33 = UPPER21.index((2, 2))
    dc = m.dc21.copy()
    dc[q33] *= a
    dc[q33][inside] *= 1.0 + 0.02 * rng.uniform(-1, 1, size=int(inside.sum()))
    drho = m.drho * b
    drho[inside] *= 1.0 + 0.02 * rng.uniform(-1, 1, size=int(inside.sum()))
    return Model(m.shape, m.h, m.C0, m.rho0, dc, drho, m.freqs, m.sources, m.tol, "config4-observed")


# the nine orthorhombic stiffnesses (Voigt index pairs) and their packed upper-triangle positions
ORTHO_PAIRS = ((0, 0), (1, 1), (2, 2), (3, 3), (4, 4), (5, 5), (0, 1), (0, 2), (1, 2))


def packed_index(I, J):
    I, J = min(I, J), max(I, J)
    return I * 6 - I * (I - 1) // 2 + (J - I)


def ortho_background(seed=4, rel=0.10):
    """Orthorhombic background: the nine orthorhombic constants of config 2's VTI medium scaled by
    1 + rel * U(-1, 1) (seed), redrawn until the 6x6 is positive definite.  Returns (C0, rho0)."""
    base = vti_from_thomsen(**VTI_CFG2)
    rng = np.random.default_rng(seed)
    while True:
        f = 1.0 + rel * rng.uniform(-1.0, 1.0, size=9)
        C = np.zeros((6, 6))
        for q, (I, J) in enumerate(ORTHO_PAIRS):
            C[I, J] = C[J, I] = base[I, J] * f[q]
        if np.linalg.eigvalsh(C).min() > 0.0:
            return C, VTI_CFG2["rho"]


CONFIG5_GRIDS = ((256, 6.0), (192, 8.0), (128, 12.0))


def config5(n=256, seed=4, freqs=(10.0, 70.0 / 3.0, 110.0 / 3.0, 50.0), corr_len=40.0, layers=3):
    """The large uneven batch: grid n^3 of (256, 192, 128) with h = 6, 8, 12 m (1536 m cubes);
    orthorhombic background (seed 4); contrast = three z layers, each scaling the nine orthorhombic
    constants and rho by 1 + 0.1 U(-1, 1), times 1 + 0.08 g (0.04 g on rho), g Gaussian random fields
    with correlation length 40 m; 6 elementary moment tensors at the centre x 4 frequencies 10-50 Hz;
    tol 1e-6.  (At 50 Hz the 12 m grid has fewer than 4 cells per S wavelength.)"""
    h = dict(CONFIG5_GRIDS)[n]
    C0, rho0 = ortho_background(seed)
    rng = np.random.default_rng(1000 * seed + n)
    lf = 1.0 + 0.10 * rng.uniform(-1.0, 1.0, size=(layers, 10))
    layer = np.minimum((np.arange(n) * layers) // n, layers - 1)
    dc = np.zeros((21, n, n, n))
    for q, (I, J) in enumerate(ORTHO_PAIRS):
        g = gaussian_random_fields(rng, 1, n, h, corr_len)[0]
        dc[packed_index(I, J)] = C0[I, J] * (lf[layer, q][:, None, None] * (1.0 + 0.08 * g) - 1.0)
    g = gaussian_random_fields(rng, 1, n, h, corr_len)[0]
    drho = rho0 * (lf[layer, 9][:, None, None] * (1.0 + 0.04 * g) - 1.0)
    m = n // 2
    sources = [(np.eye(6)[J], (m, m, m)) for J in range(6)]
    return Model((n, n, n), h, C0, rho0, dc, drho, list(map(float, freqs)), sources, 1e-6, f"config5_{n}")


def random_field(shape, seed, complex_=True):
    """Seeded standard-normal test field [3, N3, N2, N1] (complex by default)."""
    rng = np.random.default_rng(seed)
    n1, n2, n3 = shape
    re = rng.standard_normal((3, n3, n2, n1))
    if not complex_:
        return re
    return re + 1j * rng.standard_normal((3, n3, n2, n1))


def random_medium(shape, seed, rel=0.1, h=10.0, aniso_background=False):
    """Small general-anisotropic test medium: every one of the 21 contrast values per cell drawn at random."""
    rng = np.random.default_rng(seed)
    n1, n2, n3 = shape
    rho0 = 2400.0
    C0 = vti_from_thomsen(**VTI_CFG2) if aniso_background else iso_C(3000.0, 1730.0, rho0)
    scale = np.abs(pack21(C0)).max()
    dc = rel * scale * rng.uniform(-1.0, 1.0, size=(21, n3, n2, n1))
    drho = rel * rho0 * rng.uniform(-1.0, 1.0, size=(n3, n2, n1))
    return Model(tuple(shape), h, C0, rho0, dc, drho, [15.0], [], 1e-8, "random")


# The paper's Model 2 (heterogeneous VTI model, Table 2): stiffnesses in GPa per layer as printed, in the
# order (c11, c33, c55 = c44, c66, c13); the layers are 108, 104 and 108 m thick from the top (z = 0).
PAPER_MODEL2_LAYERS = ((34.0, 26.5, 10.4, 11.7, 6.9),     # top VTI layer
                       (29.05, 29.05, 10.0, 10.0, 9.05),  # isotropic layer
                       (33.8, 21.9, 6.0, 12.0, 8.0))      # bottom VTI layer
PAPER_MODEL2_THICKNESS = (108.0, 104.0, 108.0)


def paper_model2(n=128, h=2.5, freqs=(50.0,), background="middle"):
    """The paper's Model 2 on an n^3 grid of spacing h (128 x 2.5 m = 320 m as printed): cell (i, j, k) takes
    the layer containing its centre depth k h; density 2500 everywhere; an explosion at the grid centre (in
    the middle layer).  Background: "middle", the isotropic middle layer (zero contrast there, usable with
    the closed-form isotropic tensor); or "mean", the thickness-weighted mean of the three VTI stiffnesses,
    itself VTI, for the anisotropic background tensor.  The stiffness inside the box is the same either way;
    outside it, where the background continues, the two choices are different media."""
    rho = 2500.0
    layers = [vti_C(*(1e9 * np.array(p))) for p in PAPER_MODEL2_LAYERS]
    if background == "middle":
        C0 = layers[1]
    elif background == "mean":
        w = np.array(PAPER_MODEL2_THICKNESS) / sum(PAPER_MODEL2_THICKNESS)
        C0 = sum(wi * C for wi, C in zip(w, layers))
    else:
        raise ValueError("background must be 'middle' or 'mean'")
    bounds = np.cumsum(PAPER_MODEL2_THICKNESS)
    depth = np.arange(n) * h
    which = np.searchsorted(bounds, depth, side="right").clip(0, 2)
    dc = np.zeros((21, n, n, n))
    for L, C in enumerate(layers):
        dc[:, which == L] = pack21(C - C0)[:, None, None, None]
    m = n // 2
    return Model((n, n, n), h, C0, rho, dc, np.zeros((n, n, n)), list(map(float, freqs)), [(EXPLOSION, (m, m, m))],
                 1e-6, "paper_model2")
