"""Pins of the oracle's time-domain synthesis: the closed-form Ricker spectrum against quadrature of the
wavelet, the inverse transform against the time shift it must produce (a pure delay e^{i w tau} turns the
wavelet into the wavelet delayed by tau), the convention of the oracle's frequency-domain fields (a
constant-velocity travel time), and the frequency truncation's error bound."""

import numpy as np

from oracle import synthesis as syn


def test_ricker_spectrum_matches_quadrature():
    fp, ts = 60.0, 0.025
    t = np.linspace(-0.2, 0.25, 180001)
    r = syn.ricker(t, fp, ts)
    for f in (5.0, 30.0, 60.0, 90.0, 150.0):
        w = 2 * np.pi * f
        quad = np.trapezoid(r * np.exp(1j * w * t), t)
        assert abs(quad - syn.ricker_spectrum(w, fp, ts)) < 1e-9 * abs(syn.ricker_spectrum(2 * np.pi * fp, fp, 0))
    # peak of |S| at the peak frequency, zero at w = 0
    f = np.linspace(1, 200, 1991)
    assert abs(f[np.argmax(np.abs(syn.ricker_spectrum(2 * np.pi * f, fp, 0)))] - fp) < 0.2
    assert syn.ricker_spectrum(0.0, fp, ts) == 0


def test_synthesis_of_a_delay_is_the_delayed_wavelet():
    """U(w) = S(w) e^{i w tau}: the trace is ricker(t - tau) (sampled; the wavelet is negligible at both
    ends of the record, so the periodic wrap-around is below the truncation error)."""
    fp, ts, dt, nt = 60.0, 0.025, 0.0003, 800
    tau = 0.04
    k = syn.synthesis_indices(nt, dt, fp, 1e-9)
    w = 2 * np.pi * k / (nt * dt)
    U = syn.ricker_spectrum(w, fp, ts) * np.exp(1j * w * tau)
    tr = syn.traces(U, k, nt, dt)
    want = syn.ricker(np.arange(nt) * dt, fp, ts + tau)
    assert np.abs(tr - want).max() < 1e-7
    # a sign error in the exponent would advance the wavelet instead
    assert np.abs(syn.traces(np.conj(U), k, nt, dt) - want).max() > 0.5


def test_truncation_error_is_bounded_by_the_threshold():
    fp, ts, dt, nt = 60.0, 0.025, 0.0003, 800
    full = syn.synthesis_indices(nt, dt, fp, 0.0)
    w = lambda k: 2 * np.pi * k / (nt * dt)
    ref = syn.traces(syn.ricker_spectrum(w(full), fp, ts), full, nt, dt)
    for eps in (1e-3, 1e-6):
        k = syn.synthesis_indices(nt, dt, fp, eps)
        assert len(k) < len(full)
        tr = syn.traces(syn.ricker_spectrum(w(k), fp, ts), k, nt, dt)
        # each dropped term is below eps times the largest; their sum bounds the error
        dropped = np.setdiff1d(full, k)
        bound = 2 * np.sum(np.abs(syn.ricker_spectrum(w(dropped), fp, 0))) / (nt * dt)
        assert np.abs(tr - ref).max() <= bound + 1e-12


def test_oracle_fields_use_the_same_time_convention():
    """The oracle's far field of a point force carries e^{+i w r / beta} (outgoing under e^{-i w t}); through
    the synthesis its S-wave arrives at t = ts + r / beta, not before the source time."""
    from oracle import green
    fp, ts, dt, nt = 60.0, 0.025, 0.0003, 800
    alpha, beta, rho, r = 3000.0, 1700.0, 2400.0, 150.0
    k = syn.synthesis_indices(nt, dt, fp, 1e-9)
    w = 2 * np.pi * k / (nt * dt)
    d = np.array([[0.0, r, 0.0]])       # transverse to a unit force along x: only the S wave reaches it
    G = np.array([green.green_exact(d, wk, alpha, beta, rho)[0, 0, 0] for wk in w])
    tr = syn.traces(syn.ricker_spectrum(w, fp, ts) * G, k, nt, dt)
    t_peak = np.argmax(np.abs(tr)) * dt
    assert abs(t_peak - (ts + r / beta)) < 3 * dt
