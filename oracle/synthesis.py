"""TEST INFRASTRUCTURE ONLY: time-domain seismograms from the frequency-domain solutions (the paper's
frequency loop up to Nyquist followed by an inverse Fourier transform; Ricker wavelet of its Tables 1 and 3).

Conventions (those of the whole oracle): time dependence e^{-i w t}, so a signal s(t) has the spectrum
S(w) = int s(t) e^{i w t} dt and s(t) = (1/2 pi) int S(w) e^{-i w t} dw.  A real medium gives
u(-w) = conj u(w), so only w >= 0 is solved.  Sampling t_n = n dt (n < nt) makes the spectrum periodic with
frequencies w_k = 2 pi k / (nt dt), k = 0 .. nt/2.
"""

import numpy as np


def ricker(t, fp, ts):
    """Ricker wavelet of peak frequency fp delayed by ts: (1 - 2 a (t - ts)^2) exp(-a (t - ts)^2), a = pi^2 fp^2."""
    a = (np.pi * fp) ** 2
    tt = np.asarray(t, dtype=np.float64) - ts
    return (1.0 - 2.0 * a * tt * tt) * np.exp(-a * tt * tt)


def ricker_spectrum(w, fp, ts):
    """Its spectrum int r(t) e^{i w t} dt = (4 sqrt(pi) w^2 / wp^3) exp(-w^2 / wp^2) e^{i w ts}, wp = 2 pi fp
    (the Gaussian integral sqrt(pi/a) e^{-w^2/4a} and its second w-derivative for the t^2 term)."""
    w = np.asarray(w, dtype=np.float64)
    wp = 2.0 * np.pi * fp
    return 4.0 * np.sqrt(np.pi) * w * w / wp ** 3 * np.exp(-(w / wp) ** 2) * np.exp(1j * w * ts)


def synthesis_indices(nt, dt, fp, eps):
    """Frequency indices k = 1 .. nt/2 whose wavelet spectrum magnitude is at least eps times its largest
    value there (the others contribute less than eps relative and are not solved).  k = 0 is excluded: the
    Ricker wavelet has no zero-frequency content."""
    k = np.arange(1, nt // 2 + 1)
    mag = np.abs(ricker_spectrum(2.0 * np.pi * k / (nt * dt), fp, 0.0))
    return k[mag >= eps * mag.max()]


def traces(U, k, nt, dt):
    """Real traces from one-sided spectra: U [len(k), ...] at w_k = 2 pi k / (nt dt) -> [..., nt] with
    u(t_n) = (1/(nt dt)) sum over all k of U_k e^{-i w_k t_n}, the negative-frequency half supplied by
    conj(U), so each 0 < k < nt/2 counts twice and k = 0 and k = nt/2 once (the latter real)."""
    U = np.asarray(U)
    k = np.asarray(k)
    n = np.arange(nt)
    out = np.zeros(U.shape[1:] + (nt,))
    for q, kk in enumerate(k):
        ph = np.exp(-2j * np.pi * (kk * n % nt) / nt)
        weight = 1.0 if (kk == 0 or 2 * kk == nt) else 2.0
        out += weight * np.real(U[q][..., None] * ph)
    return out / (nt * dt)
