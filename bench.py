#!/usr/bin/env python3
"""Benchmark of the LS displacement solver on one MI355X.

Workload (the metric's configuration): a 128^3 grid, h = 8 m, TTI stiffness (config 2's VTI tilted
30 deg about y and rotated 45 deg about z) with Gaussian random-field perturbations (8 % on all 21
stiffnesses, 4 % on density, correlation length 40 m, seed 2) over an isotropic background
(3000, 1700, 2400); 6 elementary moment tensors x 8 frequencies 5-40 Hz at the centre cell;
relative residual 1e-6 certified with the FP64 operator.

One step = the whole hot path over that batch in one library call (ls_solve_batch): the 48 moment-tensor
incident fields, then one mixed-precision solve of all 48 systems, each at its own frequency, sharing every
operator launch (FP32 operator inside Bi-CGSTAB with FP64 inner products, FP64 iterative refinement with
the FP64 operator, final FP64 true residual); systems leave the launches as they converge.  The Green's
tables for the 8 frequencies are built once before the timed region (set-up time is reported
separately).  ``value`` is LS matvecs per second over the timed steps (every operator application of
every right-hand side counts once, FP32 and FP64 alike); the timed steps replay captured graphs.

Also reported: the operator alone (c128 and c64, 1 and 6 right-hand sides), the roofline of the
dominant kernel measured with HIP events on the library's stream during one extra untimed step, the same
48 systems solved one at a time with the plain FP64 operator, and the CPU oracle's FFT-based apply timed
on the host as a baseline.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LS matvecs/s + time-to-solve (rel res 1e-6) at 128^3; HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def family_bytes(fam, n, L, sum_rhs, sum_tabs, count):
    """Algorithmic HBM bytes of the recorded launches of one kernel family (each array read or written once):
    a part per right-hand side the launches covered (sum_rhs), a part per launch (the contrast, read once
    per launch whatever its width) and a part per distinct Green's table a launch read (sum_tabs)."""
    if "." not in fam:
        return None
    name, prec = fam.rsplit(".", 1)
    sc = 16 if prec == "c128" else 8      # complex element
    sr = sc // 2                          # real element
    N = n ** 3
    xl = 3 * n * n                        # data lines of the x passes per right-hand side
    yc = 3 * n * L                        # columns of the y passes per right-hand side
    octant = (L // 2 + 1) ** 3
    per_rhs = {
        "contrast_fused": 6 * N * sc,             # u in, f out
        "contrast_fused_T": 9 * N * sc,           # g in, y in, out
        "contrast_strain_stress": 9 * N * sc,     # u in, tau out
        "contrast_divergence": 12 * N * sc,       # tau, u in, f out
        "fft_x_fwd": xl * (n + L) * sc,
        "fft_y_fwd": yc * (n + L) * sc,
        "fft_z_green": 2 * 3 * n * L * L * sc,
        "fft_y_inv": yc * (L + n) * sc,
        "fft_x_inv_epi": xl * (L + 2 * n) * sc,   # work in, u in, Au out
        "fft_x_inv_rv": xl * (L + 3 * n) * sc,    # also r^ in (r^H v fused)
        "fft_x_inv_ts": xl * (L + 2 * n) * sc,    # t^H s uses u = s, already read
        "fft_x_inv_conv": xl * (L + n) * sc,
    }
    per_launch = {"contrast_fused": 22 * N * sr, "contrast_fused_T": 22 * N * sr,
                  "contrast_strain_stress": 21 * N * sr, "contrast_divergence": N * sr}
    per_table = {"fft_z_green": 6 * octant * sc}
    if name not in per_rhs:
        return None
    return per_rhs[name] * sum_rhs + per_launch.get(name, 0) * count + per_table.get(name, 0) * sum_tabs


FP_VECTOR_PEAK_TFLOPS = 78.6   # 256 CUs x 64 lanes x 2 flops (FMA) x 2.4 GHz, FP32 without packed math, and FP64


def kernel_flops(fam, n1, n2, n3, L1, L2, L3, nrhs):
    """Algorithmic flops of z-pass launches covering nrhs right-hand sides in all: per (k_x, k_y) column and
    right-hand side, a forward and an inverse length-L3 FFT of three components at the conventional
    5 L log2 L each, plus the complex 3 x 3 multiply (9 complex multiply-adds, 8 flops each) at every k_z."""
    if not fam.startswith("fft_z_green"):
        return None
    import math
    per_column = 3 * 2 * 5 * L3 * math.log2(L3) + 72 * L3
    return per_column * L1 * L2 * nrhs


def split_contrast():
    """True when the two-kernel contrast (strain/stress, then divergence) is selected instead of the fused one."""
    return os.environ.get("LS_CONTRAST", "") == "split"


def apply_bytes(n, prec, nrhs):
    """Algorithmic bytes of one LS matvec of nrhs right-hand sides at one frequency (L = 2N): the sum over
    its kernels."""
    L = 2 * n
    contrast = ("contrast_strain_stress", "contrast_divergence") if split_contrast() else ("contrast_fused",)
    return sum(family_bytes(f + "." + prec, n, L, nrhs, 1, 1) for f in
               contrast + ("fft_x_fwd", "fft_y_fwd", "fft_z_green", "fft_y_inv", "fft_x_inv_epi"))


# the sources each kernel family is compiled from (a change to any of them voids its counter figures)
FAMILY_SOURCES = {"fft_": ("common.h", "fft_core.h", "fft_reg.h", "fft.hip"),
                  "contrast_": ("common.h", "fft_reg.h", "contrast.hip")}


def file_hash(name):
    """sha256 (first 16 hex digits) of one HIP source file of the library."""
    import hashlib
    with open(os.path.join(ROOT, "paper_2301_12836_amd", "csrc", name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(family, n, L, rhs_per_launch, R=6):
    """HBM bytes per launch of a kernel family, from the committed rocprofv3 counter summary of R-right-hand-
    side applies at one frequency: the counters' ratio to that launch's algorithmic bytes, times the
    algorithmic bytes of a launch of the given average width.  (None, reason) when the summary is missing
    or any source the family is compiled from differs from the one the counters were taken with."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_config3_apply.txt")
    srcs = next((v for k, v in FAMILY_SOURCES.items() if family.startswith(k)), None)
    if srcs is None or not os.path.exists(path):
        return None, "no counter summary for this family"
    lines = open(path).read().splitlines()
    recorded = {p[1]: p[2] for p in (ln.split() for ln in lines) if len(p) == 3 and p[0] == "file_sha256"}
    if any(recorded.get(f) != file_hash(f) for f in srcs):
        return None, "the kernel sources changed since the counters were taken"
    for ln in lines:
        parts = ln.split()
        if len(parts) == 3 and parts[0] == "traffic" and parts[1] == family:
            counted = float(parts[2])
            alg = family_bytes(family, n, L, R, 1, 1)
            per_launch = family_bytes(family, n, L, rhs_per_launch, 1, 1)
            return round(counted / alg * per_launch), (
                f"FETCH_SIZE + WRITE_SIZE of a {R}-right-hand-side launch: {counted:.4g} B against {alg:.4g} B "
                f"algorithmic (ratio {counted / alg:.3f}), scaled to {rhs_per_launch:.2f} right-hand sides per launch")
    return None, "family not in the counter summary"


def time_applies(torch, ctx, u, reps, warmup=5):
    """Median and interquartile range (s) of single applies, each bracketed by HIP events on the stream
    the context runs on (torch's current stream)."""
    import numpy as np
    out = torch.empty_like(u)
    for _ in range(warmup):
        ctx.apply(u, 0, out=out)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        ctx.apply(u, 0, out=out)
        b.record()
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev]) * 1e-3
    q1, med, q3 = np.percentile(t, [25, 50, 75])
    return med, q3 - q1


def cpu_baseline(model, reps):
    """The oracle's FFT apply (FP64, scipy.fft on all host threads) on the same model at 5 Hz."""
    import numpy as np

    from oracle import operator as op
    from paper_2301_12836_amd import models
    P = op.Problem(model.shape, model.h, model.C0, model.rho0, model.dc21, model.drho, model.omegas[0])
    P.table()   # built once, not timed (like the GPU tables)
    u = models.random_field(model.shape, 0)
    t0 = time.perf_counter()
    for _ in range(reps):
        P.apply_fft(u)
    dt = (time.perf_counter() - t0) / reps
    threads = os.cpu_count()
    try:
        threads = len(os.sched_getaffinity(0))
    except Exception:
        pass
    return {"value": 1.0 / dt, "unit": "matvecs/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} oracle FFT applies (FP64, scipy.fft workers=-1) of the 128^3 model at 5 Hz, "
                      f"one right-hand side; {dt:.2f} s each; Green's table built beforehand, untimed"}


COPY_BYTES = 1 << 30


def apply_profile(args):
    """A short run for rocprofv3: 3 batched c64 applies, 3 batched c128 applies and 3 copies of a 1 GiB
    buffer (a plain copy kernel of known size, to calibrate the FETCH_SIZE / WRITE_SIZE counters)."""
    import numpy as np
    import torch

    from paper_2301_12836_amd import lsvie, models
    model = models.config3(n=args.n)
    log(f"model built: {args.n}^3")
    nrhs = len(model.sources)
    ctx = lsvie.context_from_model(model, precision="mixed", max_rhs=nrhs, omegas=model.omegas[-1:])
    u = torch.from_numpy(np.stack([models.random_field(model.shape, s) for s in range(nrhs)])).to(ctx.device)
    for dt_ in (torch.complex64, torch.complex128):
        uu = u.to(dt_)
        out = torch.empty_like(uu)
        for _ in range(3):
            ctx.apply(uu, 0, out=out)
        torch.cuda.synchronize()
        log(f"3 applies of {nrhs} right-hand sides in {dt_}")
        del uu, out
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=ctx.device).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"3 copies of {COPY_BYTES} bytes")
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128, help="grid size (128 is the metric's workload)")
    ap.add_argument("--maxit", type=int, default=3000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--no-compare-c128", action="store_true",
                    help="skip timing the same 48 systems as sequential single-source plain c128 solves")
    ap.add_argument("--bicgstab-l", type=int, default=1,
                    help="Krylov method: 1 Bi-CGSTAB (the paper's), 2..4 BiCGSTAB(l)")
    ap.add_argument("--mode", choices=["bench", "steps", "apply-profile"], default="bench",
                    help="steps: only the warmup and timed steps (for rocprofv3 kernel traces of the solve); "
                         "apply-profile: only a few batched applies plus a copy of known size, for counter runs")
    args = ap.parse_args()
    if args.mode == "apply-profile":
        return apply_profile(args)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): sharding the independent "
              "(grid, frequency) jobs over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2301_12836_amd import lsvie, models

    t0 = time.perf_counter()
    model = models.config3(n=args.n)
    log(f"model built in {time.perf_counter() - t0:.1f} s: {model.shape}, h={model.h}, freqs={model.freqs}")
    n = args.n
    L = 2 * n
    nrhs = len(model.sources)
    nfreq = len(model.omegas)
    nsys = nrhs * nfreq
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = lsvie.context_from_model(model, precision="mixed", max_rhs=nsys, bicgstab_l=args.bicgstab_l)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"context set up in {setup_s:.2f} s ({ctx.device_bytes / 2**30:.2f} GiB on the device)")

    # the 48 systems: every moment tensor at every frequency, frequency-major
    jobs = [(0, iw, M, src, 0.0) for iw in range(nfreq) for M, src in model.sources]
    out = ctx.empty(nsys)
    outs = [out[k] for k in range(nsys)]

    def step():
        """One ls_solve_batch call: the 48 incident fields, then one mixed-precision solve of all 48 systems
        (each at its own frequency) in shared launches."""
        _, infos = lsvie.solve_batch([ctx], jobs, tol=model.tol, maxit=args.maxit, precision="mixed", outs=outs)
        mv = sum(i["matvecs"] for i in infos)
        its = [[infos[iw * nrhs + J]["iters"] for J in range(nrhs)] for iw in range(nfreq)]
        res = [max(infos[iw * nrhs + J]["rel_res_true"] for J in range(nrhs)) for iw in range(nfreq)]
        refs = [[infos[iw * nrhs + J]["refinements"] for J in range(nrhs)] for iw in range(nfreq)]
        for iw in range(nfreq):
            log(f"  {model.freqs[iw]:.0f} Hz: iterations {its[iw]}, refinements {refs[iw]}, "
                f"worst residual {res[iw]:.2e}")
        return mv, its, res

    for w in range(args.warmup):
        t0 = time.perf_counter()
        mv, its, res = step()
        torch.cuda.synchronize()
        log(f"warmup step {w}: {time.perf_counter() - t0:.2f} s, {mv} matvecs, worst residual {max(res):.2e}")

    # the timed steps run the product path as shipped: per-kernel event recording off, so every Bi-CGSTAB
    # iteration replays its captured hipGraph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_mv = 0
    for k in range(args.steps):
        mv, its, res = step()
        total_mv += mv
        log(f"step {k}: {mv} matvecs, iterations per frequency {[max(i) for i in its]}, "
            f"worst residual {max(res):.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = total_mv / elapsed
    log(f"timed {args.steps} steps: {ms_per_step:.1f} ms per step, {value:.1f} matvecs/s")
    if args.mode == "steps":
        ctx.close()
        print(json.dumps({"mode": "steps", "ms_per_step": round(ms_per_step, 2), "matvecs_per_s": round(value, 1)}),
              flush=True)
        return

    # one more step, untimed, with a HIP event pair recorded around every kernel launch on the library's
    # stream (ls_profile; the iterations then run as separate launches instead of graph replays): the
    # per-kernel table and the roofline of the dominant kernel come from it
    ctx.profile(True)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    step()
    torch.cuda.synchronize()
    profiled_ms = 1e3 * (time.perf_counter() - tp)
    prof = ctx.profile_read()
    ctx.profile(False)
    log(f"profiled step: {profiled_ms:.1f} ms (event pairs around every launch, no graph replay)")

    # error of every mixed-precision result (last timed step) against FP64 solves of the same systems to a
    # relative residual of 1e-10 (the FP64 path is the one held to the oracle at 1e-10 in the parity tests)
    b_all = ctx.empty(nsys)
    for k, (_, iw, M, src, t0_) in enumerate(jobs):
        ctx.rhs_moment(M, src, i_omega=iw, t0=t0_, out=b_all[k])
    ref, _ = ctx.solve(b_all, i_omega=[j[1] for j in jobs], tol=1e-10, maxit=args.maxit, precision="c128")
    d = (torch.linalg.vector_norm((out - ref).reshape(nsys, -1), dim=1)
         / torch.linalg.vector_norm(ref.reshape(nsys, -1), dim=1)).cpu().numpy()
    errs = [[float(d[iw * nrhs + J]) for J in range(nrhs)] for iw in range(nfreq)]
    del ref, b_all
    accuracy = {"reference": "FP64 solves of the same 48 systems to relative residual 1e-10",
                "max_rel_err": max(max(e) for e in errs),
                "per_frequency_max": [float(f"{max(e):.3g}") for e in errs]}
    log(f"mixed vs FP64 per-result relative error: max {accuracy['max_rel_err']:.2e}, per frequency "
        f"{accuracy['per_frequency_max']}")

    # roofline of the dominant kernel family during the profiled step: algorithmic bytes of its launches
    # (each launch's own width and tables) over their summed event time
    fam_rows = []
    for fam, d_ in prof.items():
        if d_["count"] == 0:
            continue
        b_ = family_bytes(fam, n, L, d_["rhs"], d_["tables"], d_["count"])
        if b_ is None:
            continue
        fam_rows.append((d_["ms"], fam, d_["count"], b_, d_["rhs"]))
    fam_rows.sort(reverse=True)
    total_prof_ms = sum(d_["ms"] for d_ in prof.values())
    kernels = {f: {"launches": c, "avg_ms": round(ms / c, 4), "rhs_per_launch": round(r / c, 2),
                   "share": round(ms / total_prof_ms, 3), "GBps": round(b_ / (ms * 1e-3) / 1e9, 1)}
               for ms, f, c, b_, r in fam_rows}
    dom_total_ms, dom, dom_count, dom_bytes_total, dom_rhs = fam_rows[0]
    dom_ms = dom_total_ms / dom_count
    dom_bytes = dom_bytes_total / dom_count
    achieved = dom_bytes_total / (dom_total_ms * 1e-3) / 1e9
    traffic, traffic_note = measured_traffic(dom, n, L, dom_rhs / dom_count)
    roofline = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_note": traffic_note,
                "bytes_per_launch": round(dom_bytes), "avg_launch_ms": round(dom_ms, 4), "launches": dom_count,
                "rhs_per_launch": round(dom_rhs / dom_count, 2)}
    log(f"dominant kernel {dom}: {dom_ms:.3f} ms avg over {dom_count} launches, {achieved:.0f} GB/s")
    # the same kernel against the vector-arithmetic peak: it is bound by its FP32 instructions, not by HBM
    roofline_alu = None
    fl = kernel_flops(dom, n, n, n, L, L, L, dom_rhs)
    if fl is not None:
        tf = fl / (dom_total_ms * 1e-3) / 1e12
        roofline_alu = {"kernel": dom, "bound": "alu", "achieved": round(tf, 2), "peak": FP_VECTOR_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(tf / FP_VECTOR_PEAK_TFLOPS, 4),
                        "flops_per_launch": fl / dom_count}
        log(f"  {tf:.1f} TFLOP/s algorithmic ({tf / FP_VECTOR_PEAK_TFLOPS:.2f} of the vector peak)")

    # the operator alone
    rates = {}
    for prec, dt_ in (("c128", torch.complex128), ("c64", torch.complex64)):
        for r in (1, nrhs):
            u = torch.from_numpy(np.stack([models.random_field(model.shape, s) for s in range(r)])).to(
                ctx.device).to(dt_)
            per, iqr = time_applies(torch, ctx, u, 50)
            rates[f"{prec}_x{r}"] = {"matvecs_per_s": round(r / per, 1), "ms_per_apply": round(per * 1e3, 3),
                                     "iqr_ms": round(iqr * 1e3, 3),
                                     "GBps_algorithmic": round(apply_bytes(n, prec, r) / per / 1e9, 1)}
            del u
    log(f"apply rates: {json.dumps(rates)}")
    ctx.close()
    del out, outs

    seq = None
    if not args.no_compare_c128:
        # the same 48 systems, one source per call, plain FP64 operator (outside the timed steps)
        ctx1 = lsvie.context_from_model(model, precision="c128", max_rhs=1)
        b1, x1 = ctx1.empty(), ctx1.empty()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mv1 = 0
        for iw in range(len(model.omegas)):
            for M, src in model.sources:
                ctx1.rhs_moment(M, src, i_omega=iw, out=b1)
                _, infos = ctx1.solve(b1, i_omega=iw, tol=model.tol, maxit=args.maxit, precision="c128", out=x1)
                mv1 += infos[0]["matvecs"]
        torch.cuda.synchronize()
        seq_s = time.perf_counter() - t0
        seq = {"time_s": round(seq_s, 3), "matvecs": mv1, "speedup_of_batched_mixed": round(seq_s / (ms_per_step / 1e3), 2)}
        log(f"sequential plain c128: {seq_s:.2f} s for the same systems ({mv1} matvecs)")
        ctx1.close()

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle baseline")
        cpu = cpu_baseline(model, args.cpu_reps)
        log(f"cpu baseline: {cpu['value']:.3f} matvecs/s on {cpu['cores']} threads")

    result = {
        "metric": METRIC, "value": round(value, 2), "unit": "matvecs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64/f64", "data": "synthetic",
        "config": {"workload": f"{n}^3 h=8 m TTI + Gaussian random fields, 6 moment tensors x 8 frequencies "
                               f"5-40 Hz, batched mixed-precision BiCGSTAB to rel res 1e-6",
                   "grid": n, "rhs": nrhs * len(model.omegas), "tol": model.tol, "bicgstab_l": args.bicgstab_l},
        "time_to_solve_s": round(ms_per_step / 1e3, 3),
        "setup_s": round(setup_s, 3),
        "time_to_solve_incl_setup_s": round(ms_per_step / 1e3 + setup_s, 3),
        "iterations_per_frequency": [max(i) for i in its],
        "worst_rel_res_true": max(res),
        "accuracy": accuracy,
        "apply": rates,
        "sequential_c128": seq,
        "kernels": kernels,
        "kernel_timing": "HIP events on the library's stream around every launch, during one extra untimed step "
                         f"({round(profiled_ms, 1)} ms; the timed steps replay graphs without events)",
        "roofline": roofline,
        "roofline_alu": roofline_alu,
        "cpu_baseline": cpu,
    }
    print(json.dumps(result), flush=True)
    report_children()


def report_children():
    """Log any process this benchmark started that is still alive (there should be none)."""
    try:
        import psutil
        kids = psutil.Process().children(recursive=True)
    except Exception as e:  # pragma: no cover - psutil missing
        log(f"child process check unavailable: {e}")
        return
    if kids:
        log("processes still alive at exit: " + ", ".join(f"{k.pid} {k.name()}" for k in kids))
    else:
        log("no child processes left at exit")


if __name__ == "__main__":
    main()
