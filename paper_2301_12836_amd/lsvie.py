"""ctypes binding of the HIP LS library (include/ls.h): argument marshalling only.

Every computation runs in the library's HIP kernels on the GPU; this module only converts
torch tensors to device pointers and checks shapes.  If the shared library has not been built,
loading fails loudly (there is no CPU fallback).

The module-level functions carry the C names (``ls_setup``, ``ls_apply``, ``ls_apply_noalloc``, ``ls_apply_c64``,
``ls_rhs_moment``, ``ls_rhs_force``, ``ls_solve``, ``ls_solve_multi``, ``ls_solve_moment``, ``ls_solve_force``,
``ls_solve_batch``, ``ls_strain``, ``ls_apply_T``, ``ls_convolve``, ``ls_solve_T``,
``ls_grad_contrast``, ``ls_grad``, ``ls_sample``, ``ls_synthesize``, ``ls_residual_history``, ``ls_profile``,
``ls_profile_read``, ``ls_device_bytes``, ``ls_kernel_variants``, ``ls_kernel_schedule``, ``ls_destroy``); ``Context`` wraps
them for convenience, and ``solve_batch`` wraps ``ls_solve_batch`` over several contexts.
"""

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "liblsvie.so")

LS_OK = 0
LS_ERR_ARG = -1
LS_ERR_OOM = -2
LS_ERR_HIP = -3
LS_ERR_BREAKDOWN = -4
LS_ERR_NOT_CONVERGED = -5
LS_ERR_NONFINITE = -6
LS_ERR_STATE = -7
LS_PREC_C128 = 0
LS_PREC_MIXED = 1
LS_GREEN_EXACT = 0
LS_GREEN_PAPER_SUM = 1
LS_GREEN_ANISO = 2
GREEN_MODES = {"exact": LS_GREEN_EXACT, "paper_sum": LS_GREEN_PAPER_SUM, "aniso": LS_GREEN_ANISO}
LS_FLAG_NO_GRAPH = 1
LS_FLAG_AUTOTUNE = 2
LS_PRECOND_NONE = 0
LS_PRECOND_BLOCK_JACOBI = 1
PRECONDS = {None: LS_PRECOND_NONE, "none": LS_PRECOND_NONE, "block_jacobi": LS_PRECOND_BLOCK_JACOBI}
PASS_NAMES = ("x_fwd", "y_fwd", "z_green", "y_inv", "x_inv")

ERROR_NAMES = {LS_ERR_ARG: "LS_ERR_ARG", LS_ERR_OOM: "LS_ERR_OOM", LS_ERR_HIP: "LS_ERR_HIP",
               LS_ERR_BREAKDOWN: "LS_ERR_BREAKDOWN", LS_ERR_NOT_CONVERGED: "LS_ERR_NOT_CONVERGED",
               LS_ERR_NONFINITE: "LS_ERR_NONFINITE", LS_ERR_STATE: "LS_ERR_STATE"}

EXPORTED = ("ls_setup", "ls_destroy", "ls_apply", "ls_apply_noalloc", "ls_apply_c64", "ls_rhs_moment", "ls_rhs_force", "ls_solve",
            "ls_solve_moment", "ls_solve_multi", "ls_solve_force", "ls_strain", "ls_set_contrast", "ls_precond_blocks", "ls_apply_T", "ls_convolve",
            "ls_solve_T", "ls_grad_contrast", "ls_grad", "ls_solve_batch", "ls_sample", "ls_synthesize", "ls_residual_history",
            "ls_profile", "ls_profile_read", "ls_device_bytes", "ls_kernel_variants", "ls_kernel_schedule", "ls_contrast_format", "ls_last_error")


class LsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("h", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("green_mode", ctypes.c_int), ("max_rhs", ctypes.c_int),
                ("flags", ctypes.c_int), ("taper", ctypes.c_int), ("bicgstab_l", ctypes.c_int),
                ("precond", ctypes.c_int), ("reserved", ctypes.c_int * 1)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("matvecs", ctypes.c_int), ("refinements", ctypes.c_int),
                ("status", ctypes.c_int), ("rel_res", ctypes.c_double), ("rel_res_true", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Job(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_int), ("i_omega", ctypes.c_int), ("M", ctypes.c_double * 6),
                ("src", ctypes.c_int * 3), ("t0", ctypes.c_double), ("u_out", ctypes.c_void_p)]


_lib = None


def library_path():
    return LIB_PATH


def load():
    """Load liblsvie.so (raises if it is missing: build it with paper_2301_12836_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run `python -m paper_2301_12836_amd.build`); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    sig = {
        "ls_setup": (I, [ctypes.POINTER(Grid), dp, D, P, P, dp, I, ctypes.POINTER(Options), P,
                         ctypes.POINTER(P)]),
        "ls_destroy": (None, [P]),
        "ls_set_contrast": (I, [P, P, P]),
        "ls_precond_blocks": (I, [P, I, P]),
        "ls_apply": (I, [P, I, P, P, I]),
        "ls_apply_noalloc": (I, [P, I, P, P, I]),
        "ls_apply_c64": (I, [P, I, P, P, I]),
        "ls_rhs_moment": (I, [P, I, dp, ip, D, P]),
        "ls_rhs_force": (I, [P, I, dp, ip, P]),
        "ls_solve": (I, [P, I, P, I, D, I, I, P, P, ctypes.POINTER(Info)]),
        "ls_solve_multi": (I, [P, ip, P, I, D, I, I, P, P, ctypes.POINTER(Info)]),
        "ls_solve_moment": (I, [P, I, dp, ip, D, D, I, I, P, P, ctypes.POINTER(Info)]),
        "ls_strain": (I, [P, P, P, I]),
        "ls_apply_T": (I, [P, I, P, P, I]),
        "ls_convolve": (I, [P, I, P, P, I]),
        "ls_solve_T": (I, [P, I, P, I, D, I, I, P, P, ctypes.POINTER(Info)]),
        "ls_grad_contrast": (I, [P, I, P, P, I, P, P]),
        "ls_grad": (I, [P, I, P, P, I, ip, dp, P, P, dp]),
        "ls_solve_batch": (I, [ctypes.POINTER(P), I, ctypes.POINTER(Job), I, D, I, I, ctypes.POINTER(Info)]),
        "ls_sample": (I, [P, P, I, ip, I, P]),
        "ls_residual_history": (I, [P, I, dp, I]),
        "ls_synthesize": (I, [P, P, ip, I, I, I, D, D, D, P]),
        "ls_solve_force": (I, [P, I, dp, ip, D, I, I, P, ctypes.POINTER(Info)]),
        "ls_profile": (I, [P, I]),
        "ls_profile_read": (I, [P, ctypes.c_char_p, ip, dp, ctypes.POINTER(ctypes.c_longlong), I]),
        "ls_device_bytes": (ctypes.c_longlong, [P]),
        "ls_kernel_variants": (I, [P, ip]),
        "ls_kernel_schedule": (I, [P, ip]),
        "ls_contrast_format": (I, [P]),
        "ls_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(code):
    if code != LS_OK:
        raise LsError(code, load().ls_last_error().decode())
    return code


def _dbl(a, n):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
    if a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _int3(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(3))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def storage_overlaps(a, b):
    """True when the memory of tensors a and b (contiguous) intersects."""
    na, nb = a.numel() * a.element_size(), b.numel() * b.element_size()
    x, y = a.data_ptr(), b.data_ptr()
    return na > 0 and nb > 0 and x < y + nb and y < x + na


def check_buffer(t, shape, dtype, device, name="out"):
    """Return a caller-supplied buffer unchanged once it is known to have exactly the given shape, dtype
    and device and to be contiguous; raise ValueError otherwise.  The library writes through a plain
    pointer, sized by the grid and the number of right-hand sides, so a buffer of another element
    type or shape would be written past its end."""
    if t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if not t.is_contiguous() or t.is_conj() or t.is_neg():
        raise ValueError(f"{name} must be a contiguous tensor without lazy conjugate or negative bits")
    return t


# ------------------------------------------------------------------------------------------
# C-named entry points (torch tensors in, plain pointers to the library)

def ls_setup(shape, h, C0, rho0, dC, drho, omegas, precision=LS_PREC_C128, green_mode=LS_GREEN_EXACT,
             max_rhs=1, stream=None, flags=0, taper=0, bicgstab_l=1, precond=LS_PRECOND_NONE):
    """dC, drho: contiguous float64 CUDA tensors [21, N3, N2, N1] and [N3, N2, N1]; returns a handle."""
    lib = load()
    g = Grid((ctypes.c_int * 3)(*[int(v) for v in shape]), float(h))
    opt = Options(int(precision), int(green_mode), int(max_rhs), int(flags), int(taper), int(bicgstab_l),
                  int(precond), (ctypes.c_int * 1)())
    c0, c0p = _dbl(C0, 36)
    om, omp = _dbl(omegas, len(np.atleast_1d(omegas)))
    out = ctypes.c_void_p()
    _check(lib.ls_setup(ctypes.byref(g), c0p, float(rho0), _ptr(dC), _ptr(drho), omp, len(om), ctypes.byref(opt),
                        ctypes.c_void_p(stream or 0), ctypes.byref(out)))
    return out


def ls_destroy(ctx):
    load().ls_destroy(ctx)


def ls_set_contrast(ctx, dC, drho):
    return _check(load().ls_set_contrast(ctx, _ptr(dC), _ptr(drho)))


def ls_precond_blocks(ctx, i_omega, minv):
    """minv: contiguous complex128 CUDA tensor [9, N3, N2, N1] (inverse block entry (a, b) at [3 a + b])."""
    return _check(load().ls_precond_blocks(ctx, int(i_omega), _ptr(minv)))


def ls_apply(ctx, i_omega, u, Au, n_rhs):
    return _check(load().ls_apply(ctx, int(i_omega), _ptr(u), _ptr(Au), int(n_rhs)))


def ls_apply_noalloc(ctx, i_omega, u, Au, n_rhs):
    return _check(load().ls_apply_noalloc(ctx, int(i_omega), _ptr(u), _ptr(Au), int(n_rhs)))


def ls_apply_c64(ctx, i_omega, u, Au, n_rhs):
    return _check(load().ls_apply_c64(ctx, int(i_omega), _ptr(u), _ptr(Au), int(n_rhs)))


def ls_rhs_moment(ctx, i_omega, M, src, t0, b):
    m, mp = _dbl(M, 6)
    s, sp = _int3(src)
    return _check(load().ls_rhs_moment(ctx, int(i_omega), mp, sp, float(t0), _ptr(b)))


def ls_rhs_force(ctx, i_omega, F, cell, b):
    f, fp = _dbl(F, 3)
    s, sp = _int3(cell)
    return _check(load().ls_rhs_force(ctx, int(i_omega), fp, sp, _ptr(b)))


def ls_solve(ctx, i_omega, b, n_rhs, tol, maxit, precision, x0, u_out, raise_on_error=True):
    infos = (Info * int(n_rhs))()
    code = load().ls_solve(ctx, int(i_omega), _ptr(b), int(n_rhs), float(tol), int(maxit), int(precision),
                           _ptr(x0), _ptr(u_out), infos)
    if raise_on_error:
        _check(code)
    return code, [i.as_dict() for i in infos]


def ls_solve_multi(ctx, i_omega, b, n_rhs, tol, maxit, precision, x0, u_out, raise_on_error=True):
    """i_omega: one frequency index per system (sequence of n_rhs ints)."""
    iw = np.ascontiguousarray(np.asarray(i_omega, dtype=np.int32).reshape(int(n_rhs)))
    infos = (Info * int(n_rhs))()
    code = load().ls_solve_multi(ctx, iw.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _ptr(b), int(n_rhs),
                                 float(tol), int(maxit), int(precision), _ptr(x0), _ptr(u_out), infos)
    if raise_on_error:
        _check(code)
    return code, [i.as_dict() for i in infos]


def ls_solve_moment(ctx, i_omega, M, src, t0, tol, maxit, precision, x0, u_out, raise_on_error=True):
    m, mp = _dbl(M, 6)
    s, sp = _int3(src)
    info = Info()
    code = load().ls_solve_moment(ctx, int(i_omega), mp, sp, float(t0), float(tol), int(maxit), int(precision),
                                  _ptr(x0), _ptr(u_out), ctypes.byref(info))
    if raise_on_error:
        _check(code)
    return code, info.as_dict()


def ls_solve_force(ctx, i_omega, F, cell, tol, maxit, precision, u_out, raise_on_error=True):
    f, fp = _dbl(F, 3)
    s, sp = _int3(cell)
    info = Info()
    code = load().ls_solve_force(ctx, int(i_omega), fp, sp, float(tol), int(maxit), int(precision), _ptr(u_out),
                                 ctypes.byref(info))
    if raise_on_error:
        _check(code)
    return code, info.as_dict()


def ls_strain(ctx, u, eps, n_rhs):
    return _check(load().ls_strain(ctx, _ptr(u), _ptr(eps), int(n_rhs)))


def ls_apply_T(ctx, i_omega, y, ATy, n_rhs):
    return _check(load().ls_apply_T(ctx, int(i_omega), _ptr(y), _ptr(ATy), int(n_rhs)))


def ls_convolve(ctx, i_omega, f, out, n_rhs):
    return _check(load().ls_convolve(ctx, int(i_omega), _ptr(f), _ptr(out), int(n_rhs)))


def ls_solve_T(ctx, i_omega, b, n_rhs, tol, maxit, precision, x0, x_out, raise_on_error=True):
    infos = (Info * int(n_rhs))()
    code = load().ls_solve_T(ctx, int(i_omega), _ptr(b), int(n_rhs), float(tol), int(maxit), int(precision),
                             _ptr(x0), _ptr(x_out), infos)
    if raise_on_error:
        _check(code)
    return code, [i.as_dict() for i in infos]


def ls_grad_contrast(ctx, i_omega, u, mu, n_rhs, g_dC, g_drho):
    return _check(load().ls_grad_contrast(ctx, int(i_omega), _ptr(u), _ptr(mu), int(n_rhs), _ptr(g_dC),
                                          _ptr(g_drho)))


def ls_grad(ctx, i_omega, u, lam_bar, n_rhs, g_dC, g_drho, src=None, t0=None):
    """Returns g_M as a numpy [n_rhs, 6] array when src (cells [n_rhs, 3]) is given, else None."""
    if src is None:
        _check(load().ls_grad(ctx, int(i_omega), _ptr(u), _ptr(lam_bar), int(n_rhs), None, None, _ptr(g_dC),
                              _ptr(g_drho), None))
        return None
    cells = np.ascontiguousarray(np.asarray(src, dtype=np.int32).reshape(int(n_rhs), 3))
    times = np.ascontiguousarray(np.broadcast_to(np.asarray(0.0 if t0 is None else t0, dtype=np.float64),
                                                 (int(n_rhs),)))
    gM = np.zeros((int(n_rhs), 6), dtype=np.float64)
    _check(load().ls_grad(ctx, int(i_omega), _ptr(u), _ptr(lam_bar), int(n_rhs),
                          cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                          times.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(g_dC), _ptr(g_drho),
                          gM.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return gM


def ls_solve_batch(ctxs, jobs, tol, maxit, precision, raise_on_error=True):
    """ctxs: context handles; jobs: sequence of Job.  Returns (code, [info dict per job])."""
    handles = (ctypes.c_void_p * len(ctxs))(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in ctxs])
    arr = (Job * max(len(jobs), 1))(*jobs)
    infos = (Info * max(len(jobs), 1))()
    code = load().ls_solve_batch(handles, len(ctxs), arr, len(jobs), float(tol), int(maxit), int(precision), infos)
    if raise_on_error:
        _check(code)
    return code, [infos[i].as_dict() for i in range(len(jobs))]


def _ints(a, shape):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(shape))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def ls_sample(ctx, u, n_rhs, rec, out):
    r, rp = _ints(rec, (-1, 3))
    return _check(load().ls_sample(ctx, _ptr(u), int(n_rhs), rp, len(r), _ptr(out)))


def ls_synthesize(ctx, spectra, k, n_trace, nt, dt, fp, ts, traces):
    kk, kp = _ints(k, (-1,))
    return _check(load().ls_synthesize(ctx, _ptr(spectra), kp, len(kk), int(n_trace), int(nt), float(dt),
                                       float(fp), float(ts), _ptr(traces)))


def ls_residual_history(ctx, rhs):
    """numpy array of the relative residual after each iteration of right-hand side rhs in the last solve."""
    lib = load()
    n = lib.ls_residual_history(ctx, int(rhs), None, 0)
    if n < 0:
        _check(n)
    out = np.zeros(n, dtype=np.float64)
    if n:
        _check(min(0, lib.ls_residual_history(ctx, int(rhs), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n)))
    return out


def ls_profile(ctx, enable):
    return _check(load().ls_profile(ctx, int(bool(enable))))


def ls_profile_read(ctx, n_max=64):
    """{family: {"count", "ms", "rhs", "tables"}}: launches, summed event time, summed right-hand sides and
    summed distinct Green's tables over the recorded launches of each kernel family."""
    names = ctypes.create_string_buffer(64 * n_max)
    counts = (ctypes.c_int * n_max)()
    ms = (ctypes.c_double * n_max)()
    units = (ctypes.c_longlong * (2 * n_max))()
    nf = load().ls_profile_read(ctx, names, counts, ms, units, n_max)
    if nf < 0:
        _check(nf)
    out = {}
    for k in range(min(nf, n_max)):
        name = names.raw[64 * k:64 * k + 64].split(b"\0", 1)[0].decode()
        out[name] = {"count": counts[k], "ms": ms[k], "rhs": units[2 * k], "tables": units[2 * k + 1]}
    return out


def ls_contrast_format(ctx):
    k = load().ls_contrast_format(ctx)
    if k < 0:
        _check(k)
    return k


def ls_kernel_variants(ctx):
    v = (ctypes.c_int * 10)()
    _check(load().ls_kernel_variants(ctx, v))
    return {prec: {PASS_NAMES[q]: ("fourstep", "stockham")[v[5 * p + q]] for q in range(5)}
            for p, prec in enumerate(("c128", "c64"))}


def ls_kernel_schedule(ctx):
    v = (ctypes.c_int * 4)()
    _check(load().ls_kernel_schedule(ctx, v))
    return {prec: {"xy_chunk": v[p], "wide_y_tiles": bool(v[2 + p])} for p, prec in enumerate(("c128", "c64"))}


def ls_device_bytes(ctx):
    return int(load().ls_device_bytes(ctx))


# ------------------------------------------------------------------------------------------
# convenience wrapper


class Context:
    """One grid + medium + frequency set on one GPU (owns the library context)."""

    def __init__(self, shape, h, C0, rho0, dc21, drho, omegas, precision="c128", green_mode="exact", max_rhs=1,
                 device="cuda:0", graphs=True, autotune=False, taper=0, bicgstab_l=1, precond=None):
        """precond: None or "block_jacobi" (right point-block Jacobi preconditioning of every Bi-CGSTAB solve)."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the LS library runs only on the GPU")
        self.torch = torch
        self.device = torch.device(device)
        self.shape = tuple(int(v) for v in shape)
        self.h = float(h)
        n1, n2, n3 = self.shape
        self.field_shape = (3, n3, n2, n1)
        self.max_rhs = int(max_rhs)
        self.omegas = list(np.atleast_1d(np.asarray(omegas, dtype=np.float64)))
        self.mixed = precision == "mixed"
        dc = torch.as_tensor(np.asarray(dc21, dtype=np.float64)).reshape(21, n3, n2, n1).to(self.device).contiguous()
        dr = torch.as_tensor(np.asarray(drho, dtype=np.float64)).reshape(n3, n2, n1).to(self.device).contiguous()
        self.stream = torch.cuda.current_stream(self.device)
        self.handle = ls_setup(self.shape, h, C0, rho0, dc, dr, self.omegas,
                               LS_PREC_MIXED if self.mixed else LS_PREC_C128,
                               GREEN_MODES[green_mode], max_rhs,
                               self.stream.cuda_stream,
                               (0 if graphs else LS_FLAG_NO_GRAPH) | (LS_FLAG_AUTOTUNE if autotune else 0),
                               int(taper), int(bicgstab_l), PRECONDS[precond])
        del dc, dr

    def close(self):
        if self.handle is not None:
            ls_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_contrast(self, dc21, drho):
        """Replace the contrast (numpy or torch; [21, N3, N2, N1] and [N3, N2, N1], float64)."""
        torch = self.torch
        n1, n2, n3 = self.shape
        dc = torch.as_tensor(dc21, dtype=torch.float64).reshape(21, n3, n2, n1).to(self.device).contiguous()
        dr = torch.as_tensor(drho, dtype=torch.float64).reshape(n3, n2, n1).to(self.device).contiguous()
        ls_set_contrast(self.handle, dc, dr)

    def precond_blocks(self, i_omega=0):
        """Inverse diagonal blocks of the block-Jacobi preconditioner: complex128 [N3, N2, N1, 3, 3]."""
        torch = self.torch
        out = torch.empty((9,) + self.field_shape[1:], dtype=torch.complex128, device=self.device)
        ls_precond_blocks(self.handle, i_omega, out)
        return out.permute(1, 2, 3, 0).reshape(self.field_shape[1:] + (3, 3))

    # helpers
    def _field(self, t, dtype=None):
        torch = self.torch
        t = torch.as_tensor(t, device=self.device)
        if dtype is not None:
            t = t.to(dtype)
        if t.dtype not in (torch.complex128, torch.complex64):
            t = t.to(torch.complex128)
        # lazy conjugate / negative views keep the original data behind data_ptr(): materialise them
        t = t.resolve_conj().resolve_neg().contiguous()
        if t.shape[-4:] != self.field_shape:
            raise ValueError(f"field shape {tuple(t.shape)} does not end in {self.field_shape}")
        nrhs = 1 if t.dim() == 4 else int(np.prod(t.shape[:-4]))
        return t, nrhs

    def _check(self, t, shape, dtype, name="out"):
        return check_buffer(t, shape, dtype, self._device_index(), name)

    def _device_index(self):
        d = self.device
        return d if d.index is not None else self.torch.device(d.type, self.torch.cuda.current_device())

    def _out(self, out, like):
        """A fresh output like the (already converted) input, or the caller's buffer once checked (it must
        not share memory with the input: the library reads the input while it writes the output)."""
        if out is None:
            return self.torch.empty_like(like)
        self._check(out, like.shape, like.dtype)
        if storage_overlaps(out, like):
            raise ValueError("out shares memory with the input")
        return out

    def empty(self, nrhs=None, dtype=None):
        torch = self.torch
        shape = self.field_shape if nrhs is None else (nrhs,) + self.field_shape
        return torch.empty(shape, dtype=dtype or torch.complex128, device=self.device)

    def apply(self, u, i_omega=0, out=None):
        u, nrhs = self._field(u)
        out = self._out(out, u)
        if u.dtype == self.torch.complex64:
            ls_apply_c64(self.handle, i_omega, u, out, nrhs)
        else:
            ls_apply(self.handle, i_omega, u, out, nrhs)
        return out

    def rhs_moment(self, M, src, i_omega=0, t0=0.0, out=None):
        out = self.empty() if out is None else self._check(out, self.field_shape, self.torch.complex128)
        ls_rhs_moment(self.handle, i_omega, M, src, t0, out)
        return out

    def rhs_force(self, F, cell, i_omega=0, out=None):
        out = self.empty() if out is None else self._check(out, self.field_shape, self.torch.complex128)
        ls_rhs_force(self.handle, i_omega, F, cell, out)
        return out

    def solve(self, b, i_omega=0, tol=1e-8, maxit=2000, precision=None, x0=None, out=None, raise_on_error=True):
        """Solve A u = b for the fields b; i_omega is one frequency index for all of them, or a sequence with
        one per field (then every system runs at its own frequency in the same launches)."""
        b, nrhs = self._field(b, self.torch.complex128)
        if x0 is not None:
            x0, _ = self._field(x0, self.torch.complex128)
        out = self._out(out, b)
        prec = LS_PREC_MIXED if (precision or ("mixed" if self.mixed else "c128")) == "mixed" else LS_PREC_C128
        if np.ndim(i_omega) == 0:
            code, infos = ls_solve(self.handle, i_omega, b, nrhs, tol, maxit, prec, x0, out, raise_on_error)
        else:
            code, infos = ls_solve_multi(self.handle, i_omega, b, nrhs, tol, maxit, prec, x0, out, raise_on_error)
        return out, infos

    def solve_moment(self, M, src, i_omega=0, t0=0.0, tol=1e-8, maxit=2000, precision=None, x0=None, out=None,
                     raise_on_error=True):
        """One moment-tensor source M (Voigt 6) at cell src: incident field and solve in one library call,
        from the initial guess x0 (None for zero; it may be out itself)."""
        out = self.empty() if out is None else self._check(out, self.field_shape, self.torch.complex128)
        if x0 is not None and x0 is not out:
            x0, _ = self._field(x0, self.torch.complex128)
        prec = LS_PREC_MIXED if (precision or ("mixed" if self.mixed else "c128")) == "mixed" else LS_PREC_C128
        code, info = ls_solve_moment(self.handle, i_omega, M, src, t0, tol, maxit, prec, x0, out, raise_on_error)
        return out, info

    def apply_T(self, y, i_omega=0, out=None):
        y, nrhs = self._field(y, self.torch.complex128)
        out = self._out(out, y)
        ls_apply_T(self.handle, i_omega, y, out, nrhs)
        return out

    def convolve(self, f, i_omega=0, out=None):
        f, nrhs = self._field(f, self.torch.complex128)
        out = self._out(out, f)
        ls_convolve(self.handle, i_omega, f, out, nrhs)
        return out

    def solve_T(self, b, i_omega=0, tol=1e-8, maxit=2000, precision=None, x0=None, out=None, raise_on_error=True):
        b, nrhs = self._field(b, self.torch.complex128)
        if x0 is not None:
            x0, _ = self._field(x0, self.torch.complex128)
        out = self._out(out, b)
        prec = LS_PREC_MIXED if (precision or ("mixed" if self.mixed else "c128")) == "mixed" else LS_PREC_C128
        code, infos = ls_solve_T(self.handle, i_omega, b, nrhs, tol, maxit, prec, x0, out, raise_on_error)
        return out, infos

    def grad_contrast(self, u, mu, i_omega=0, g_dC=None, g_drho=None):
        """Accumulate dJ/d(dC) [21, N3, N2, N1] and dJ/d(drho) [N3, N2, N1] (float64, on the device)."""
        torch = self.torch
        u, nrhs = self._field(u, torch.complex128)
        mu, nrhs2 = self._field(mu, torch.complex128)
        if nrhs != nrhs2:
            raise ValueError("u and mu must hold the same number of fields")
        if g_dC is None:
            g_dC = torch.zeros((21,) + self.field_shape[1:], dtype=torch.float64, device=self.device)
        else:
            self._check(g_dC, (21,) + self.field_shape[1:], torch.float64, "g_dC")
        if g_drho is None:
            g_drho = torch.zeros(self.field_shape[1:], dtype=torch.float64, device=self.device)
        else:
            self._check(g_drho, self.field_shape[1:], torch.float64, "g_drho")
        ls_grad_contrast(self.handle, i_omega, u, mu, nrhs, g_dC, g_drho)
        return g_dC, g_drho

    def solve_force(self, F, cell, i_omega=0, tol=1e-8, maxit=2000, precision=None, out=None,
                    raise_on_error=True):
        out = self.empty() if out is None else self._check(out, self.field_shape, self.torch.complex128)
        prec = LS_PREC_MIXED if (precision or ("mixed" if self.mixed else "c128")) == "mixed" else LS_PREC_C128
        code, info = ls_solve_force(self.handle, i_omega, F, cell, tol, maxit, prec, out, raise_on_error)
        return out, info

    def grad(self, u, lam_bar, i_omega=0, src=None, t0=None, g_dC=None, g_drho=None):
        """Gradient of one frequency from forward fields u and adjoint solutions lam_bar (A^T lam_bar =
        conj(P^H r)): accumulates g_dC [21, N3, N2, N1] and g_drho [N3, N2, N1] (float64, on the device) and
        returns (g_dC, g_drho, g_M) with g_M a numpy [n_rhs, 6] array when src is given, else None."""
        torch = self.torch
        u, nrhs = self._field(u, torch.complex128)
        lam_bar, nrhs2 = self._field(lam_bar, torch.complex128)
        if nrhs != nrhs2:
            raise ValueError("u and lam_bar must hold the same number of fields")
        if g_dC is None:
            g_dC = torch.zeros((21,) + self.field_shape[1:], dtype=torch.float64, device=self.device)
        else:
            self._check(g_dC, (21,) + self.field_shape[1:], torch.float64, "g_dC")
        if g_drho is None:
            g_drho = torch.zeros(self.field_shape[1:], dtype=torch.float64, device=self.device)
        else:
            self._check(g_drho, self.field_shape[1:], torch.float64, "g_drho")
        gM = ls_grad(self.handle, i_omega, u, lam_bar, nrhs, g_dC, g_drho, src=src, t0=t0)
        return g_dC, g_drho, gM

    def sample(self, u, receivers):
        """Receiver samples [n_rhs, n_rec, 3] (complex128, on the device) of fields u at cells [n_rec, 3]."""
        u, nrhs = self._field(u, self.torch.complex128)
        nrec = int(np.asarray(receivers).reshape(-1, 3).shape[0])
        out = self.torch.empty((nrhs, nrec, 3), dtype=self.torch.complex128, device=self.device)
        ls_sample(self.handle, u, nrhs, receivers, out)
        return out

    def synthesize(self, spectra, k, nt, dt, fp=0.0, ts=0.0):
        """Traces [n_trace, nt] (float64, on the device) from one-sided spectra [n_freq, n_trace] at the
        frequency indices k (w_k = 2 pi k / (nt dt)), times the Ricker wavelet (fp, ts) when fp > 0."""
        torch = self.torch
        spectra = torch.as_tensor(spectra, device=self.device).to(torch.complex128).resolve_conj().contiguous()
        if spectra.dim() != 2 or spectra.shape[0] != len(np.atleast_1d(k)):
            raise ValueError("spectra must be [n_freq, n_trace] with one row per frequency index")
        traces = torch.empty((spectra.shape[1], int(nt)), dtype=torch.float64, device=self.device)
        ls_synthesize(self.handle, spectra, k, spectra.shape[1], nt, dt, fp, ts, traces)
        return traces

    def strain(self, u):
        u, nrhs = self._field(u, self.torch.complex128)
        eps = self.torch.empty(u.shape[:-4] + (6,) + self.field_shape[1:], dtype=u.dtype, device=self.device)
        ls_strain(self.handle, u, eps, nrhs)
        return eps

    def residual_history(self, rhs=0):
        return ls_residual_history(self.handle, rhs)

    def profile(self, enable=True):
        ls_profile(self.handle, enable)

    def profile_read(self):
        return ls_profile_read(self.handle)

    @property
    def contrast_format(self):
        """Values per cell of the packed contrast the fused kernel reads: 9 (orthotropic pattern) or 21."""
        return ls_contrast_format(self.handle)

    @property
    def kernel_variants(self):
        return ls_kernel_variants(self.handle)

    @property
    def kernel_schedule(self):
        return ls_kernel_schedule(self.handle)

    @property
    def device_bytes(self):
        return ls_device_bytes(self.handle)


def solve_batch(contexts, jobs, tol=1e-8, maxit=2000, precision="c128", raise_on_error=True, outs=None):
    """Solve moment-tensor jobs over several contexts (grids may differ) in one library call.

    jobs: sequence of (context index, frequency index, M[6], (i, j, k), t0).  Returns (fields, infos):
    one complex128 [3, N3, N2, N1] tensor per job on its context's device (new ones, or the caller's outs,
    one per job, each checked), and the per-job info."""
    if outs is not None and len(outs) != len(jobs):
        raise ValueError("outs must hold one field per job")
    new_outs, arr = [], []
    for k, (ci, iw, M, src, t0) in enumerate(jobs):
        ctx = contexts[ci]
        out = ctx.empty() if outs is None else ctx._check(outs[k], ctx.field_shape, ctx.torch.complex128)
        new_outs.append(out)
        arr.append(Job(int(ci), int(iw), (ctypes.c_double * 6)(*np.asarray(M, dtype=np.float64).reshape(6)),
                       (ctypes.c_int * 3)(*[int(v) for v in src]), float(t0), out.data_ptr()))
    prec = LS_PREC_MIXED if precision == "mixed" else LS_PREC_C128
    code, infos = ls_solve_batch([c.handle for c in contexts], arr, tol, maxit, prec, raise_on_error)
    return new_outs, infos


def context_from_model(model, precision="c128", max_rhs=1, green_mode="exact", device="cuda:0", omegas=None,
                       graphs=True, autotune=False, taper=0, bicgstab_l=1, precond=None):
    return Context(model.shape, model.h, model.C0, model.rho0, model.dc21, model.drho,
                   model.omegas if omegas is None else omegas, precision=precision, green_mode=green_mode,
                   max_rhs=max_rhs, device=device, graphs=graphs, autotune=autotune, taper=taper,
                   bicgstab_l=bicgstab_l, precond=precond)
