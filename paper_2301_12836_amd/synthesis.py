"""Time-domain seismograms: the frequency loop up to Nyquist, receiver spectra and the inverse transform
(the workflow of the paper's comparisons with finite differences; Ricker wavelet of its Tables 1 and 3).

Time dependence e^{-i w t}; w_k = 2 pi k / (nt dt).  Only the frequencies whose wavelet spectrum reaches
eps of its largest value below Nyquist are solved (the others add less than eps relative each); a real
medium gives u(-w) = conj u(w), so negative frequencies are not solved.  Frequencies are taken in chunks:
each chunk gets one context (its Green's tables live only while the chunk is solved) and one
``ls_solve_batch`` call over its (frequency, source) systems; the receiver samples of every solution stay
on the device, and ``ls_synthesize`` forms the traces.  All field work runs in the HIP library.
"""

import numpy as np

from . import lsvie


def frequency_indices(nt, dt, fp, eps):
    """k in 1 .. nt/2 with |S(w_k)| >= eps max |S| for the Ricker wavelet of peak frequency fp."""
    k = np.arange(1, nt // 2 + 1)
    x = (k / (nt * dt)) / fp
    mag = x * x * np.exp(-x * x)
    return k[mag >= eps * mag.max()]


def seismograms(model, sources, receivers, nt, dt, fp, ts, eps=1e-6, tol=1e-8, precision="mixed", chunk=16,
                maxit=3000, taper=0, device="cuda:0", green_mode="exact", bicgstab_l=1, raise_on_error=True):
    """Traces [n_src, n_rec, 3, nt] (float64, on the device) of the displacement at the receiver cells
    [n_rec, 3] for the moment-tensor sources [(M6, (i, j, k), t0)], each with the Ricker time function of
    peak frequency fp delayed by ts; returns (traces, k, infos) with k the solved frequency indices and
    infos the per-system solver reports.  green_mode and bicgstab_l are the context options of the same
    names (the background's own anisotropic tensor; BiCGSTAB(l) for the high frequencies).  With
    raise_on_error=False a system that stops short of tol keeps its best iterate and reports its status in
    infos instead of raising."""
    import torch
    k = frequency_indices(nt, dt, fp, eps)
    receivers = np.asarray(receivers, dtype=np.int64).reshape(-1, 3)
    nsrc, nrec = len(sources), len(receivers)
    spectra, ctx, infos = None, None, []
    for c0 in range(0, len(k), chunk):
        kc = k[c0:c0 + chunk]
        if ctx is not None:
            ctx.close()
        ctx = lsvie.context_from_model(model, precision=precision, max_rhs=nsrc, omegas=2 * np.pi * kc / (nt * dt),
                                       taper=taper, device=device, green_mode=green_mode, bicgstab_l=bicgstab_l)
        if spectra is None:
            spectra = torch.empty((len(k), nsrc, nrec, 3), dtype=torch.complex128, device=ctx.device)
        jobs = [(0, i, M, src, t0) for i in range(len(kc)) for (M, src, t0) in sources]
        outs, inf = lsvie.solve_batch([ctx], jobs, tol=tol, maxit=maxit, precision=precision,
                                      raise_on_error=raise_on_error)
        infos.extend(inf)
        for i in range(len(kc)):
            spectra[c0 + i] = ctx.sample(torch.stack(outs[i * nsrc:(i + 1) * nsrc]), receivers)
        del outs
    traces = ctx.synthesize(spectra.reshape(len(k), -1), k, nt, dt, fp, ts).reshape(nsrc, nrec, 3, nt)
    ctx.close()
    return traces, k, infos
